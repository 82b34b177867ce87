/*
 * dsdna_oracle.c -- plain, slow FP64 CPU oracle for one Langevin time step of
 * the single-nucleotide dsDNA model of Fosado, Michieletto, Allan, Brackley,
 * Henrich and Marenduzzo, "A single nucleotide resolution model for
 * large-scale simulations of double stranded DNA" (arXiv:1608.03722).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the tests, the smoke check of the entry module and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper with
 * the HIP library, and the HIP library never calls it.
 *
 * Every function follows the passage of the paper cited above it, in the
 * order the paper states it, with no blocking, fusion or reordering.  Where
 * the paper is silent the reading used is named in the comment (readings are
 * listed with their reasons in the design notes of the repository).
 *
 * Pins: every function is checked by the tests against closed forms, finite
 * differences of its own energy, invariants, brute force or a library
 * routine.  Parity unpinned: whether the readings of what the paper leaves
 * open (unit masses, friction 1, the noise distribution, the hydrogen-bond
 * depth convention, the planarity triple, the bubble rule, the tether and
 * the placement of the pulling force) are the ones of the authors' own
 * input scripts, which are not published; the paper gives no worked
 * numerical example of a force or a step.
 *
 * Conventions
 *   - reduced units of Table 3: sigma = 1 nm, epsilon = k_B T, tau_Br.
 *   - replica r holds n_bp[r] base pairs; nucleotide (strand s, bp n) of
 *     replica r has index off[r] + 2 n + s (base-pair-major interleaving).
 *   - a nucleotide is the rigid bead+patch body of Sec. 2: bead and patch sit
 *     on the body axis u, a distance ell apart, around the centre of mass R.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ types */

typedef struct {
    /* Table 2 (Appendix A) */
    double K1, R0, eps_bb, sig_bb; /* backbone FENE + its own WCA core     */
    double K2, r0_hb, rc_hb;       /* hydrogen bond (truncated harmonic)   */
    double eps, sig_s, sig_x;      /* steric WCA: same-strand sigma, cross */
    double K3, d_dih;              /* dihedral, phase d in radians         */
    double K4, lam, r0_m;          /* Morse stacking                       */
    double K5, a0;                 /* planarity harmonic, alpha0 radians   */
    double K6;                     /* Kratky-Porod bending                 */
    /* Sec. 2: the rigid nucleotide */
    double ell, m_bead, m_patch;
    /* Appendix A: Langevin equation and time step */
    double gamma, kT, dt;
    uint64_t seed;
    int32_t noise_kind;            /* 0 Gaussian (Box-Muller), 1 uniform   */
    int32_t ssdna_rule;            /* Sec. 5 rule for bubbles > 2 bp       */
    int32_t hb_depth_convention;   /* 0: prefactor K2/(2(r0-rc)^2)         */
    int32_t fene_clamp;            /* 1: hold 1 - r^2/R0^2 at >= 0.1 (a
                                      reading for overstretched bonds)     */
    int32_t dihedral_damping;      /* 1: dihedral x sin^3 of both bond
                                      angles (a reading, see below)        */
    int32_t planarity_both;        /* 1: a second planarity angle per step
                                      (the mirrored triple, see below)     */
} orc_params;

typedef struct {
    int32_t n_rep;
    const int32_t *n_bp;      /* [n_rep]                                   */
    const double *box;        /* [n_rep][6]: lo x,y,z then hi x,y,z        */
    const uint8_t *periodic;  /* [n_rep][3]                                */
    const double *pull;       /* [n_rep][3]: force on the last base pair   */
    const double *torque;     /* [n_rep][3]: torque on the last base pair  */
    const uint8_t *tether;    /* [n_rep]: first bp anchored + bead wall    */
    const double *wall_z;     /* [n_rep]: wall plane z                     */
    const double *k2_scale;   /* [n_rep]: multiplies K2                    */
    const uint8_t *circular;  /* [n_rep]: closed ring (bp n_bp-1 bonded to
                                 bp 0), may be NULL                         */
    const double *k2_bp;      /* [sum n_bp]: multiplies K2 of each base
                                 pair (sequence, Sec. 5), may be NULL       */
} orc_system;

typedef struct {
    int64_t n_nt;
    double *R, *u, *V, *L;    /* [n_nt][3] body state                      */
    double *fb, *fp;          /* [n_nt][3] total site forces of last eval  */
    int64_t step;
    int32_t has_f;            /* 1 when fb/fp hold the forces at `step`   */
    int32_t pad;
} orc_state;

enum { T_EXCL = 0, T_BOND, T_STACK, T_HBOND, T_TWIST, T_PLANAR, T_BEND, T_EXT, NTERM };

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EBOND = 4, ORC_ENAN = 5, ORC_EWALL = 7 };

/* -------------------------------------------------------- vector helpers */

typedef struct { double x, y, z; } v3;

static v3 v3_ld(const double *p) { v3 r = {p[0], p[1], p[2]}; return r; }
static void v3_st(double *p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
static void v3_acc(double *p, v3 a) { p[0] += a.x; p[1] += a.y; p[2] += a.z; }
static v3 v3_add(v3 a, v3 b) { v3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static v3 v3_sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static v3 v3_mul(v3 a, double s) { v3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double v3_dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 v3_cross(v3 a, v3 b)
{
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static double v3_len(v3 a) { return sqrt(v3_dot(a, a)); }

/* ------------------------------------------------------------- topology */

static int64_t total_nt(const orc_system *sys)
{
    int64_t n = 0;
    for (int r = 0; r < sys->n_rep; ++r) n += 2 * (int64_t)sys->n_bp[r];
    return n;
}

static int64_t rep_offset(const orc_system *sys, int r)
{
    int64_t off = 0;
    for (int q = 0; q < r; ++q) off += 2 * (int64_t)sys->n_bp[q];
    return off;
}

static int64_t nt_index(int64_t off, int s, int64_t n) { return off + 2 * n + s; }

/* Sec. 2 / Fig. 1(d): along each strand one sterically interacting bead is
 * followed by two ghost beads.  Reading: bead (s, n) is steric iff n % 3 == 0
 * on both strands. */
static int is_steric(int64_t n) { return (n % 3) == 0; }

/* ------------------------------------------------------- rigid nucleotide */

/* Sec. 2: bead and patch 0.5 nm apart on one rigid body.  With masses m_b,
 * m_p the centre of mass R splits the axis in the ratio m_p : m_b. */
void orc_sites_from_bodies(const orc_params *P, int64_t n_nt, const double *R, const double *u,
                           double *bead, double *patch)
{
    double M = P->m_bead + P->m_patch;
    double db = P->ell * P->m_patch / M; /* |bead - R|  */
    double dp = P->ell * P->m_bead / M;  /* |patch - R| */
    for (int64_t i = 0; i < n_nt; ++i) {
        v3 Ri = v3_ld(R + 3 * i), ui = v3_ld(u + 3 * i);
        v3_st(bead + 3 * i, v3_sub(Ri, v3_mul(ui, db)));
        v3_st(patch + 3 * i, v3_add(Ri, v3_mul(ui, dp)));
    }
}

void orc_bodies_from_sites(const orc_params *P, int64_t n_nt, const double *bead,
                           const double *patch, double *R, double *u)
{
    double M = P->m_bead + P->m_patch;
    for (int64_t i = 0; i < n_nt; ++i) {
        v3 b = v3_ld(bead + 3 * i), p = v3_ld(patch + 3 * i);
        v3 d = v3_sub(p, b);
        v3 ui = v3_mul(d, 1.0 / v3_len(d));
        v3 Ri = v3_mul(v3_add(v3_mul(b, P->m_bead), v3_mul(p, P->m_patch)), 1.0 / M);
        v3_st(R + 3 * i, Ri);
        v3_st(u + 3 * i, ui);
    }
}

/* ---------------------------------------------------------- potentials */
/* Each function returns U and writes dU/dr (for pair terms). */

static const double TWO_16 = 1.12246204830937298143; /* 2^(1/6) */

/* Appendix A: truncated and shifted Lennard-Jones (WCA),
 * U = 4 eps [(s/r)^12 - (s/r)^6 + 1/4] for r < 2^(1/6) s, else 0. */
static double u_wca(double r, double eps, double sig, double *dudr)
{
    double rc = TWO_16 * sig;
    if (r >= rc) { *dudr = 0.0; return 0.0; }
    double sr6 = pow(sig / r, 6.0);
    double sr12 = sr6 * sr6;
    *dudr = -24.0 * eps * (2.0 * sr12 - sr6) / r;
    return 4.0 * eps * (sr12 - sr6 + 0.25);
}

/* Appendix A: FENE, U = -(K1 R0^2 / 2) ln[1 - (r/R0)^2] for r < R0. */
static double u_fene(double r, double K1, double R0, int clamp, double *dudr)
{
    double x = 1.0 - (r * r) / (R0 * R0);
    /* the optional hold: past 1 - r^2/R0^2 = 0.1 the argument stays at 0.1,
     * so the force grows linearly with r and the energy is capped */
    if (clamp && x < 0.1) x = 0.1;
    *dudr = K1 * r / x;
    return -0.5 * K1 * R0 * R0 * log(x);
}

/* Appendix A: Morse, U = K4 [1 - exp(-lambda (r - r0))]^2. */
static double u_morse(double r, double K4, double lam, double r0, double *dudr)
{
    double e = exp(-lam * (r - r0));
    *dudr = 2.0 * K4 * lam * e * (1.0 - e);
    return K4 * (1.0 - e) * (1.0 - e);
}

/* ------------------------------------------------------------ pair rule */

/* Sec. 2 and Table 2: WCA between beads.  Reading of the steric rule
 * (Sec. 2, Fig. 1(d)):
 *   same strand, both steric  -> sigma = sig_s (1 nm)
 *   same strand, any ghost    -> no interaction
 *   different strands         -> sigma = sig_x (0.5 nm), every bead type
 * Replicas never interact.  Returns 0 when the pair does not interact. */
static int pair_sigma(const orc_params *P, int si, int64_t ni, int sj, int64_t nj, double *sig)
{
    if (si == sj) {
        if (is_steric(ni) && is_steric(nj)) { *sig = P->sig_s; return 1; }
        return 0;
    }
    *sig = P->sig_x;
    return 1;
}

static v3 min_image(v3 d, const orc_system *sys, int r)
{
    const double *box = sys->box + 6 * r;
    const uint8_t *per = sys->periodic + 3 * r;
    double *c = &d.x;
    for (int k = 0; k < 3; ++k) {
        if (per[k]) {
            double Lk = box[3 + k] - box[k];
            c[k] -= Lk * nearbyint(c[k] / Lk);
        }
    }
    return d;
}

/* ------------------------------------------------------------- WCA pairs */

typedef struct {
    const orc_params *P;
    const orc_system *sys;
    const double *bead;
    double *fb;      /* [N][3] force on beads (T_EXCL slice) */
    double *E;       /* per replica energy of T_EXCL        */
    int64_t *pairs;  /* optional pair log (i, j), i < j     */
    int64_t n_pairs, cap_pairs;
} wca_ctx;

static void wca_pair(wca_ctx *w, int r, int64_t off, int64_t i, int64_t j)
{
    int si = (int)((i - off) & 1), sj = (int)((j - off) & 1);
    int64_t ni = (i - off) >> 1, nj = (j - off) >> 1;
    double sig;
    if (!pair_sigma(w->P, si, ni, sj, nj, &sig)) return;
    v3 d = min_image(v3_sub(v3_ld(w->bead + 3 * j), v3_ld(w->bead + 3 * i)), w->sys, r);
    double rr = v3_len(d);
    if (rr >= TWO_16 * sig) return;
    double dudr;
    double U = u_wca(rr, w->P->eps, sig, &dudr);
    v3 f = v3_mul(d, dudr / rr); /* force on i is +dU/dr * d/|d|, i.e. away from j for repulsion */
    v3_acc(w->fb + 3 * i, f);
    v3_acc(w->fb + 3 * j, v3_mul(f, -1.0));
    w->E[r] += U;
    if (w->pairs && w->n_pairs < w->cap_pairs) {
        w->pairs[2 * w->n_pairs] = i;
        w->pairs[2 * w->n_pairs + 1] = j;
    }
    w->n_pairs++;
}

/* The plain definition: every unordered bead pair of a replica (O(N^2)). */
static void wca_all_pairs(wca_ctx *w, int r, int64_t off, int64_t nnt)
{
    for (int64_t a = 0; a < nnt; ++a)
        for (int64_t b = a + 1; b < nnt; ++b) wca_pair(w, r, off, off + a, off + b);
}

/* A simple linked-cell search ("short-ranged neighbour calculations",
 * Sec. 6), checked against wca_all_pairs by the tests.  Cell edge >= the
 * largest cutoff; each unordered pair is visited once (j > i). */
static int wca_cells(wca_ctx *w, int r, int64_t off, int64_t nnt)
{
    const orc_params *P = w->P;
    double rcmax = TWO_16 * fmax(P->sig_s, P->sig_x);
    const double *box = w->sys->box + 6 * r;
    const uint8_t *per = w->sys->periodic + 3 * r;
    double lo[3], len[3];
    int64_t nc[3];
    for (int k = 0; k < 3; ++k) {
        if (per[k]) {
            lo[k] = box[k];
            len[k] = box[3 + k] - box[k];
        } else {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t a = 0; a < nnt; ++a) {
                double x = w->bead[3 * (off + a) + k];
                mn = fmin(mn, x);
                mx = fmax(mx, x);
            }
            lo[k] = mn;
            len[k] = (mx - mn) + rcmax;
        }
    }
    /* cell edge >= rcmax; enlarged until there are at most 8 cells per bead
     * (larger cells only add candidates that fail the distance test) */
    double edge = rcmax;
    for (;;) {
        for (int k = 0; k < 3; ++k) {
            nc[k] = (int64_t)floor(len[k] / edge);
            if (nc[k] < 1) nc[k] = 1;
            if (per[k] && nc[k] < 3) nc[k] = 1; /* too small for a 3-cell stencil */
        }
        if ((double)nc[0] * (double)nc[1] * (double)nc[2] <= 8.0 * (double)nnt + 64.0) break;
        edge *= 1.25;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * nnt);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * nnt * 3);
    if (!head || !next || !cid) { free(head); free(next); free(cid); return ORC_EINVAL; }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t a = nnt - 1; a >= 0; --a) {
        int64_t cc[3];
        for (int k = 0; k < 3; ++k) {
            double x = w->bead[3 * (off + a) + k] - lo[k];
            if (per[k]) x -= len[k] * floor(x / len[k]);
            int64_t c = (int64_t)floor(x / (len[k] / (double)nc[k]));
            if (c < 0) c = 0;
            if (c >= nc[k]) c = nc[k] - 1;
            cc[k] = c;
            cid[3 * a + k] = c;
        }
        int64_t flat = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
        next[a] = head[flat];
        head[flat] = a;
    }
    for (int64_t a = 0; a < nnt; ++a) {
        int64_t span[3][3];
        int ns[3];
        for (int k = 0; k < 3; ++k) {
            ns[k] = 0;
            if (nc[k] < 3) { /* every cell index along k */
                for (int64_t c = 0; c < nc[k]; ++c) span[k][ns[k]++] = c;
                continue;
            }
            for (int dk = -1; dk <= 1; ++dk) {
                int64_t c = cid[3 * a + k] + dk;
                if (per[k]) c = (c + nc[k]) % nc[k];
                else if (c < 0 || c >= nc[k]) continue;
                span[k][ns[k]++] = c;
            }
        }
        for (int iz = 0; iz < ns[2]; ++iz)
            for (int iy = 0; iy < ns[1]; ++iy)
                for (int ix = 0; ix < ns[0]; ++ix) {
                    int64_t flat = (span[2][iz] * nc[1] + span[1][iy]) * nc[0] + span[0][ix];
                    for (int64_t b = head[flat]; b >= 0; b = next[b])
                        if (b > a) wca_pair(w, r, off, off + a, off + b);
                }
    }
    free(head);
    free(next);
    free(cid);
    return ORC_OK;
}

/* ----------------------------------------------------------- angle terms */

/* Angle at vertex b between a-b and c-b.  Fills dcos/da and dcos/dc. */
static double angle_cos(v3 a, v3 b, v3 c, v3 *dca, v3 *dcc)
{
    v3 r1 = v3_sub(a, b), r2 = v3_sub(c, b);
    double l1 = v3_len(r1), l2 = v3_len(r2);
    double cs = v3_dot(r1, r2) / (l1 * l2);
    *dca = v3_sub(v3_mul(r2, 1.0 / (l1 * l2)), v3_mul(r1, cs / (l1 * l1)));
    *dcc = v3_sub(v3_mul(r1, 1.0 / (l1 * l2)), v3_mul(r2, cs / (l2 * l2)));
    return cs;
}

/* Dihedral angle of (p1, p2, p3, p4) in the IUPAC sign convention,
 * phi = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3)), b1 = p2-p1, b2 = p3-p2,
 * b3 = p4-p3, and its gradient with respect to each point following
 * Blondel & Karplus, J. Comput. Chem. 17, 1132 (1996):
 *   F = p1-p2, G = p2-p3, H = p4-p3, A = F x G, B = H x G,
 *   dphi/dp1 = -|G|/|A|^2 A,          dphi/dp4 = +|G|/|B|^2 B,
 *   dphi/dp2 = +|G|/|A|^2 A + (F.G)/(|A|^2|G|) A - (H.G)/(|B|^2|G|) B,
 *   dphi/dp3 = -|G|/|B|^2 B - (F.G)/(|A|^2|G|) A + (H.G)/(|B|^2|G|) B. */
/* sin^3 of the angle between u and w, and its gradients du, dw with respect
 * to u and w: with c the cosine, d(sin^3)/dc = -3 sin c. */
static double sin_cube(v3 u, v3 w, v3 *du, v3 *dw)
{
    double lu = v3_len(u), lw = v3_len(w);
    double c = v3_dot(u, w) / (lu * lw);
    double s2 = 1.0 - c * c;
    double s = s2 > 0.0 ? sqrt(s2) : 0.0;
    double k = -3.0 * s * c;
    *du = v3_mul(v3_sub(v3_mul(w, 1.0 / (lu * lw)), v3_mul(u, c / (lu * lu))), k);
    *dw = v3_mul(v3_sub(v3_mul(u, 1.0 / (lu * lw)), v3_mul(w, c / (lw * lw))), k);
    return s2 * s;
}

static double dihedral(v3 p1, v3 p2, v3 p3, v3 p4, v3 g[4])
{
    v3 b1 = v3_sub(p2, p1), b2 = v3_sub(p3, p2), b3 = v3_sub(p4, p3);
    v3 n1 = v3_cross(b1, b2), n2 = v3_cross(b2, b3);
    double phi = atan2(v3_len(b2) * v3_dot(b1, n2), v3_dot(n1, n2));
    v3 F = v3_sub(p1, p2), G = v3_sub(p2, p3), H = v3_sub(p4, p3);
    v3 A = v3_cross(F, G), B = v3_cross(H, G);
    double AA = v3_dot(A, A), BB = v3_dot(B, B), lG = v3_len(G);
    double FG = v3_dot(F, G), HG = v3_dot(H, G);
    v3 tA = v3_mul(A, lG / AA), tB = v3_mul(B, lG / BB);
    v3 sA = v3_mul(A, FG / (AA * lG)), sB = v3_mul(B, HG / (BB * lG));
    g[0] = v3_mul(tA, -1.0);
    g[3] = tB;
    g[1] = v3_sub(v3_add(tA, sA), sB);
    g[2] = v3_add(v3_sub(v3_mul(tB, -1.0), sA), sB);
    return phi;
}

/* ----------------------------------------------------------- open mask */

/* Sec. 2 / Appendix A: the hydrogen bond breaks beyond r_c.  A base pair is
 * "open" when the distance between its two patches exceeds r_c.  Sec. 5: a
 * bubble is a run of consecutive open base pairs; the ssDNA rule acts on
 * bubbles larger than two base pairs.  Writes in_bubble[n] = 1 for every bp
 * of a maximal open run of length >= 3. */
static void bubble_mask(const uint8_t *open, int64_t nbp, uint8_t *in_bubble)
{
    int64_t n = 0;
    while (n < nbp) {
        if (!open[n]) { in_bubble[n] = 0; ++n; continue; }
        int64_t e = n;
        while (e < nbp && open[e]) ++e;
        uint8_t big = (e - n) >= 3;
        for (int64_t k = n; k < e; ++k) in_bubble[k] = big;
        n = e;
    }
}

/* The same on a ring, where bp nbp-1 and bp 0 are neighbours: runs are
 * cyclic, and a ring with every base pair open is one bubble. */
static void bubble_mask_ring(const uint8_t *open, int64_t nbp, uint8_t *in_bubble)
{
    int64_t c = 0;
    while (c < nbp && open[c]) ++c;
    if (c == nbp) {
        for (int64_t k = 0; k < nbp; ++k) in_bubble[k] = nbp >= 3;
        return;
    }
    /* walk once round the ring from the closed base pair c */
    int64_t k = 1;
    in_bubble[c] = 0;
    while (k < nbp) {
        int64_t n = (c + k) % nbp;
        if (!open[n]) { in_bubble[n] = 0; ++k; continue; }
        int64_t e = k;
        while (e < nbp && open[(c + e) % nbp]) ++e;
        uint8_t big = (e - k) >= 3;
        for (int64_t q = k; q < e; ++q) in_bubble[(c + q) % nbp] = big;
        k = e;
    }
}

/* ---------------------------------------------------------------- forces */

/*
 * Conservative + external site forces, split by term, and energies per
 * replica and term, at the given site positions.
 *   split:           1 -> f_bead, f_patch are [NTERM][n_nt][3], one slice per
 *                    term; 0 -> [n_nt][3], all terms summed
 *   f_bead, f_patch: zeroed here, may not be NULL
 *   energy:          [n_rep][NTERM]   (zeroed here), may be NULL
 *   open_out:        [sum n_bp] open flag per base pair, may be NULL
 *   use_cells:       0 -> all pairs (the plain definition), 1 -> cell search
 * Returns ORC_OK, ORC_EBOND (backbone stretched to r >= R0, where the FENE
 * energy is infinite) or ORC_EWALL (a bead on or behind the anchoring wall);
 * *err_id then holds the first offending nucleotide.
 */
int orc_forces(const orc_params *P, const orc_system *sys, const double *bead,
               const double *patch, int use_cells, int split, double *f_bead, double *f_patch,
               double *energy, uint8_t *open_out, int64_t *err_id)
{
    int64_t N = total_nt(sys);
    int64_t tstride = split ? N : 0; /* split: one [N][3] slice per term */
    memset(f_bead, 0, sizeof(double) * (split ? NTERM : 1) * N * 3);
    memset(f_patch, 0, sizeof(double) * (split ? NTERM : 1) * N * 3);
    double *Eloc = (double *)calloc((size_t)sys->n_rep * NTERM, sizeof(double));
    int status = ORC_OK;
    if (err_id) *err_id = -1;
#define FB(t, i) (f_bead + 3 * ((int64_t)(t) * tstride + (i)))
#define FP(t, i) (f_patch + 3 * ((int64_t)(t) * tstride + (i)))
#define EN(r, t) (Eloc[(int64_t)(r) * NTERM + (t)])

    int64_t bp_base = 0;
    for (int r = 0; r < sys->n_rep; ++r) {
        int64_t nbp = sys->n_bp[r];
        int64_t off = rep_offset(sys, r);
        double k2s = sys->k2_scale ? sys->k2_scale[r] : 1.0;
        /* a ring has a backbone step from every bp n to n+1 (mod nbp) and a
         * bending triple centred on every bp; a linear chain has nbp - 1
         * steps and the triples centred on bp 1 .. nbp-2 */
        int ring = sys->circular && sys->circular[r];
        int64_t nstep = ring ? nbp : nbp - 1;
        int64_t b_first = ring ? 0 : 1, b_end = ring ? nbp : nbp - 1;

        /* --- hydrogen bond (Appendix A, U_hb): patches of (0,n) and (1,n) */
        uint8_t *open = (uint8_t *)calloc((size_t)nbp + 1, 1);
        uint8_t *inb = (uint8_t *)calloc((size_t)nbp + 1, 1);
        double K2 = P->K2 * k2s;
        double pref = (P->hb_depth_convention == 0)
                          ? K2 / (2.0 * (P->r0_hb - P->rc_hb) * (P->r0_hb - P->rc_hb))
                          : K2 / ((P->r0_hb - P->rc_hb) * (P->r0_hb - P->rc_hb));
        for (int64_t n = 0; n < nbp; ++n) {
            int64_t i = nt_index(off, 0, n), j = nt_index(off, 1, n);
            v3 d = v3_sub(v3_ld(patch + 3 * j), v3_ld(patch + 3 * i));
            double rr = v3_len(d);
            if (rr > P->rc_hb) { open[n] = 1; continue; }
            /* the base pair's own stiffness: K2 x replica scale x bp scale */
            double pn = sys->k2_bp ? pref * sys->k2_bp[bp_base + n] : pref;
            double U = pn * ((rr - P->r0_hb) * (rr - P->r0_hb) -
                             (P->rc_hb - P->r0_hb) * (P->rc_hb - P->r0_hb));
            /* -dU/dr along the unit vector from i to j, written without 1/r so
             * that r = 0 (coincident patches of the ideal helix) is regular:
             * f_i = 2 pref (r - r0)/r * d = 2 pref (1 - r0/r) d. */
            double c = (P->r0_hb == 0.0) ? 2.0 * pn : 2.0 * pn * (1.0 - P->r0_hb / rr);
            v3 f = v3_mul(d, c);
            v3_acc(FP(T_HBOND, i), f);
            v3_acc(FP(T_HBOND, j), v3_mul(f, -1.0));
            EN(r, T_HBOND) += U;
        }
        if (open_out) memcpy(open_out + bp_base, open, (size_t)nbp);
        if (P->ssdna_rule) {
            if (ring) bubble_mask_ring(open, nbp, inb);
            else bubble_mask(open, nbp, inb);
        }

        for (int s = 0; s < 2; ++s) {
            /* --- backbone: FENE + WCA(eps_bb, sig_bb) between consecutive beads */
            for (int64_t n = 0; n < nstep; ++n) {
                int64_t i = nt_index(off, s, n), j = nt_index(off, s, (n + 1) % nbp);
                v3 d = v3_sub(v3_ld(bead + 3 * j), v3_ld(bead + 3 * i));
                double rr = v3_len(d);
                if (P->fene_clamp ? rr >= 2.0 * P->R0 : rr >= P->R0) {
                    if (status == ORC_OK) { status = ORC_EBOND; if (err_id) *err_id = i; }
                    continue;
                }
                double d1, d2;
                double U = u_fene(rr, P->K1, P->R0, P->fene_clamp, &d1) + u_wca(rr, P->eps_bb, P->sig_bb, &d2);
                v3 f = v3_mul(d, (d1 + d2) / rr);
                v3_acc(FB(T_BOND, i), f);
                v3_acc(FB(T_BOND, j), v3_mul(f, -1.0));
                EN(r, T_BOND) += U;
            }
            /* --- Morse stacking between consecutive patches */
            for (int64_t n = 0; n < nstep; ++n) {
                int64_t i = nt_index(off, s, n), j = nt_index(off, s, (n + 1) % nbp);
                v3 d = v3_sub(v3_ld(patch + 3 * j), v3_ld(patch + 3 * i));
                double rr = v3_len(d);
                double dudr;
                double U = u_morse(rr, P->K4, P->lam, P->r0_m, &dudr);
                v3 f = v3_mul(d, dudr / rr);
                v3_acc(FP(T_STACK, i), f);
                v3_acc(FP(T_STACK, j), v3_mul(f, -1.0));
                EN(r, T_STACK) += U;
            }
            /* --- dihedral on (bead n, patch n, patch n+1, bead n+1),
             *     U = K3 [1 + cos(phi - d)] (Sec. 2, Appendix A) */
            for (int64_t n = 0; n < nstep; ++n) {
                if (P->ssdna_rule && inb[n] && inb[(n + 1) % nbp]) continue;
                int64_t i = nt_index(off, s, n), j = nt_index(off, s, (n + 1) % nbp);
                v3 g[4];
                double phi = dihedral(v3_ld(bead + 3 * i), v3_ld(patch + 3 * i),
                                      v3_ld(patch + 3 * j), v3_ld(bead + 3 * j), g);
                double U = P->K3 * (1.0 + cos(phi - P->d_dih));
                double dUdphi = -P->K3 * sin(phi - P->d_dih);
                if (P->dihedral_damping) {
                    /* the reading for bubbles and frayed ends: U sin^3(t1)
                     * sin^3(t2), t1 and t2 the bond angles at the two middle
                     * sites (the combined bending-torsion form of Bulacu et
                     * al., J. Chem. Theory Comput. 9, 3282 (2013)); its
                     * gradient stays finite where a bond angle reaches 0 or pi,
                     * where that of the bare dihedral diverges */
                    v3 p1 = v3_ld(bead + 3 * i), p2 = v3_ld(patch + 3 * i);
                    v3 p3 = v3_ld(patch + 3 * j), p4 = v3_ld(bead + 3 * j);
                    v3 b1 = v3_sub(p2, p1), b2 = v3_sub(p3, p2), b3 = v3_sub(p4, p3);
                    v3 d1u, d1w, d2u, d2w;
                    double S1 = sin_cube(b1, b2, &d1u, &d1w), S2 = sin_cube(b2, b3, &d2u, &d2w);
                    double S = S1 * S2;
                    v3 dS[4];
                    dS[0] = v3_mul(d1u, -S2);
                    dS[1] = v3_sub(v3_mul(v3_sub(d1u, d1w), S2), v3_mul(d2u, S1));
                    dS[2] = v3_add(v3_mul(d1w, S2), v3_mul(v3_sub(d2u, d2w), S1));
                    dS[3] = v3_mul(d2w, S1);
                    v3_acc(FB(T_TWIST, i), v3_sub(v3_mul(g[0], -dUdphi * S), v3_mul(dS[0], U)));
                    v3_acc(FP(T_TWIST, i), v3_sub(v3_mul(g[1], -dUdphi * S), v3_mul(dS[1], U)));
                    v3_acc(FP(T_TWIST, j), v3_sub(v3_mul(g[2], -dUdphi * S), v3_mul(dS[2], U)));
                    v3_acc(FB(T_TWIST, j), v3_sub(v3_mul(g[3], -dUdphi * S), v3_mul(dS[3], U)));
                    EN(r, T_TWIST) += U * S;
                    continue;
                }
                v3_acc(FB(T_TWIST, i), v3_mul(g[0], -dUdphi));
                v3_acc(FP(T_TWIST, i), v3_mul(g[1], -dUdphi));
                v3_acc(FP(T_TWIST, j), v3_mul(g[2], -dUdphi));
                v3_acc(FB(T_TWIST, j), v3_mul(g[3], -dUdphi));
                EN(r, T_TWIST) += U;
            }
            /* --- planarity: angle at patch n+1 between patch n and bead n+1,
             *     U = (K5/2)(alpha - alpha0)^2 */
            for (int64_t n = 0; n < nstep; ++n) {
                int64_t i = nt_index(off, s, n), j = nt_index(off, s, (n + 1) % nbp);
                v3 dca, dcc;
                double cs = angle_cos(v3_ld(patch + 3 * i), v3_ld(patch + 3 * j),
                                      v3_ld(bead + 3 * j), &dca, &dcc);
                if (cs > 1.0) cs = 1.0;
                if (cs < -1.0) cs = -1.0;
                double al = acos(cs);
                double U = 0.5 * P->K5 * (al - P->a0) * (al - P->a0);
                /* dU/dcos = dU/dalpha * dalpha/dcos = K5 (al - a0) * (-1/sin al) */
                double dUdc = -P->K5 * (al - P->a0) / sin(al);
                v3 fa = v3_mul(dca, -dUdc), fc = v3_mul(dcc, -dUdc);
                v3_acc(FP(T_PLANAR, i), fa);
                v3_acc(FB(T_PLANAR, j), fc);
                v3_acc(FP(T_PLANAR, j), v3_mul(v3_add(fa, fc), -1.0));
                EN(r, T_PLANAR) += U;
                if (!P->planarity_both) continue;
                /* the reading with both triples of the step: also the angle
                 * at patch n between patch n+1 and bead n (the same triple
                 * seen from the other end of the step), same potential */
                cs = angle_cos(v3_ld(patch + 3 * j), v3_ld(patch + 3 * i), v3_ld(bead + 3 * i), &dca, &dcc);
                if (cs > 1.0) cs = 1.0;
                if (cs < -1.0) cs = -1.0;
                al = acos(cs);
                U = 0.5 * P->K5 * (al - P->a0) * (al - P->a0);
                dUdc = -P->K5 * (al - P->a0) / sin(al);
                fa = v3_mul(dca, -dUdc);
                fc = v3_mul(dcc, -dUdc);
                v3_acc(FP(T_PLANAR, j), fa);
                v3_acc(FB(T_PLANAR, i), fc);
                v3_acc(FP(T_PLANAR, i), v3_mul(v3_add(fa, fc), -1.0));
                EN(r, T_PLANAR) += U;
            }
            /* --- Kratky-Porod: angle at patch n among patches n-1, n, n+1,
             *     U = K6 [1 + cos(theta)] */
            for (int64_t n = b_first; n < b_end; ++n) {
                int64_t np = (n + nbp - 1) % nbp, nn = (n + 1) % nbp;
                if (P->ssdna_rule && inb[np] && inb[n] && inb[nn]) continue;
                int64_t h = nt_index(off, s, np), i = nt_index(off, s, n),
                        j = nt_index(off, s, nn);
                v3 dca, dcc;
                double cs = angle_cos(v3_ld(patch + 3 * h), v3_ld(patch + 3 * i),
                                      v3_ld(patch + 3 * j), &dca, &dcc);
                double U = P->K6 * (1.0 + cs);
                v3 fa = v3_mul(dca, -P->K6), fc = v3_mul(dcc, -P->K6);
                v3_acc(FP(T_BEND, h), fa);
                v3_acc(FP(T_BEND, j), fc);
                v3_acc(FP(T_BEND, i), v3_mul(v3_add(fa, fc), -1.0));
                EN(r, T_BEND) += U;
            }
        }
        free(open);
        free(inb);

        /* --- excluded volume between beads (WCA, Sec. 2 rule) */
        double *Etmp = (double *)calloc((size_t)sys->n_rep, sizeof(double));
        wca_ctx w = {P, sys, bead, FB(T_EXCL, 0), Etmp, NULL, 0, 0};
        if (use_cells) wca_cells(&w, r, off, 2 * nbp);
        else wca_all_pairs(&w, r, off, 2 * nbp);
        EN(r, T_EXCL) += Etmp[r];
        free(Etmp);

        /* --- external loads (Sec. 4): anchoring wall, pull, torque */
        if (sys->tether && sys->tether[r]) {
            double zw = sys->wall_z[r];
            double rcw = TWO_16 * P->sig_s;
            for (int64_t a = 0; a < 2 * nbp; ++a) {
                int64_t i = off + a;
                double dz = bead[3 * i + 2] - zw;
                if (dz <= 0.0) {
                    if (status == ORC_OK) { status = ORC_EWALL; if (err_id) *err_id = i; }
                    continue;
                }
                if (dz >= rcw) continue;
                double dudr;
                double U = u_wca(dz, P->eps, P->sig_s, &dudr);
                FB(T_EXT, i)[2] += -dudr;
                EN(r, T_EXT) += U;
            }
        }
        if (nbp >= 1 && sys->pull) {
            /* reading: the pulling force is split equally over the two
             * patches of the last base pair (they lie on the helix axis) */
            v3 F = v3_ld(sys->pull + 3 * r);
            v3_acc(FP(T_EXT, nt_index(off, 0, nbp - 1)), v3_mul(F, 0.5));
            v3_acc(FP(T_EXT, nt_index(off, 1, nbp - 1)), v3_mul(F, 0.5));
        }
        if (nbp >= 1 && sys->torque) {
            /* reading: the torque is a couple on the two beads of the last
             * base pair about their midpoint c, f_k = G x (r_k - c) / D with
             * D = sum_k |(r_k - c) perpendicular to G|^2: zero net force and a
             * torque component exactly G along G. */
            v3 G = v3_ld(sys->torque + 3 * r);
            double G2 = v3_dot(G, G);
            if (G2 > 0.0) {
                int64_t i0 = nt_index(off, 0, nbp - 1), i1 = nt_index(off, 1, nbp - 1);
                v3 b0 = v3_ld(bead + 3 * i0), b1 = v3_ld(bead + 3 * i1);
                v3 c = v3_mul(v3_add(b0, b1), 0.5);
                v3 d0 = v3_sub(b0, c), d1 = v3_sub(b1, c);
                v3 Gh = v3_mul(G, 1.0 / sqrt(G2));
                v3 p0 = v3_sub(d0, v3_mul(Gh, v3_dot(d0, Gh)));
                v3 p1 = v3_sub(d1, v3_mul(Gh, v3_dot(d1, Gh)));
                double D = v3_dot(p0, p0) + v3_dot(p1, p1);
                if (D > 0.0) {
                    v3_acc(FB(T_EXT, i0), v3_mul(v3_cross(G, d0), 1.0 / D));
                    v3_acc(FB(T_EXT, i1), v3_mul(v3_cross(G, d1), 1.0 / D));
                }
            }
        }
        bp_base += nbp;
    }
    if (energy) memcpy(energy, Eloc, sizeof(double) * sys->n_rep * NTERM);
    free(Eloc);
#undef FB
#undef FP
#undef EN
    return status;
}

/* List of interacting WCA pairs (i < j) of replica r, for the cell-search
 * versus all-pairs test.  Returns the number of pairs (may exceed cap). */
int64_t orc_wca_pairs(const orc_params *P, const orc_system *sys, const double *bead, int r,
                      int use_cells, int64_t *pairs, int64_t cap)
{
    int64_t N = total_nt(sys);
    double *fb = (double *)calloc((size_t)N * 3, sizeof(double));
    double *E = (double *)calloc((size_t)sys->n_rep, sizeof(double));
    wca_ctx w = {P, sys, bead, fb, E, pairs, 0, cap};
    int64_t off = rep_offset(sys, r);
    if (use_cells) wca_cells(&w, r, off, 2 * (int64_t)sys->n_bp[r]);
    else wca_all_pairs(&w, r, off, 2 * (int64_t)sys->n_bp[r]);
    free(fb);
    free(E);
    return w.n_pairs;
}

/* ------------------------------------------------------------------ RNG */

/* Philox4x32-10 of Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): ten rounds of the 4-word S-box built from two
 * 32x32->64 multiplications, with the key bumped by the Weyl constants
 * between rounds. */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The same round structure on 64-bit words (Philox4x64-10), used only to pin
 * the round structure against an independent library implementation. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The six unit-variance numbers of one nucleotide at one step: components
 * (bead x, y, z, patch x, y, z).  Counter = (nucleotide id, stream<<16|call,
 * step low word, step high word); key = (seed low word, seed high word).
 * Uniforms u = (x + 1/2) 2^-32 in (0, 1).  Gaussian: Box-Muller on the pairs
 * (x0,x1), (x2,x3) of call 0 and (x0,x1) of call 1.  Uniform: sqrt(12)(u-1/2)
 * on x0..x3 of call 0 and x0, x1 of call 1. */
void orc_noise(uint64_t seed, int noise_kind, uint64_t step, int64_t id, int stream, double xi[6])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[8];
    for (int call = 0; call < 2; ++call) {
        uint32_t ctr[4] = {(uint32_t)id, ((uint32_t)stream << 16) | (uint32_t)call,
                           (uint32_t)step, (uint32_t)(step >> 32)};
        orc_philox4x32(ctr, key, w + 4 * call);
    }
    double u[6];
    for (int k = 0; k < 6; ++k) u[k] = ((double)w[k] + 0.5) * 0x1p-32;
    if (noise_kind == 1) {
        for (int k = 0; k < 6; ++k) xi[k] = sqrt(12.0) * (u[k] - 0.5);
        return;
    }
    for (int k = 0; k < 6; k += 2) {
        double rad = sqrt(-2.0 * log(u[k]));
        double ang = 2.0 * M_PI * u[k + 1];
        xi[k] = rad * cos(ang);
        xi[k + 1] = rad * sin(ang);
    }
}

/* ----------------------------------------------------------- integrator */

static int frozen(const orc_system *sys, int r, int64_t n) { return sys->tether && sys->tether[r] && n == 0; }

/* Total site forces at the state's positions: conservative and external terms
 * (orc_forces) plus the Langevin forces of Appendix A per site,
 * -gamma v_site + sqrt(2 gamma kT / dt) xi, with v_site the velocity of the
 * site on the rigid body, V + omega x (r_site - R), omega = L / I. */
static int total_forces(const orc_params *P, const orc_system *sys, orc_state *S, int use_cells,
                        int64_t *err_id)
{
    int64_t N = S->n_nt;
    double *bead = (double *)malloc(sizeof(double) * N * 3);
    double *patch = (double *)malloc(sizeof(double) * N * 3);
    double *fbt = (double *)malloc(sizeof(double) * N * 3);
    double *fpt = (double *)malloc(sizeof(double) * N * 3);
    orc_sites_from_bodies(P, N, S->R, S->u, bead, patch);
    int st = orc_forces(P, sys, bead, patch, use_cells, 0, fbt, fpt, NULL, NULL, err_id);
    double M = P->m_bead + P->m_patch;
    double I = P->m_bead * P->m_patch / M * P->ell * P->ell;
    double db = P->ell * P->m_patch / M, dp = P->ell * P->m_bead / M;
    double amp = sqrt(2.0 * P->gamma * P->kT / P->dt);
    for (int r = 0; r < sys->n_rep; ++r) {
        int64_t off = rep_offset(sys, r);
        for (int64_t a = 0; a < 2 * (int64_t)sys->n_bp[r]; ++a) {
            int64_t i = off + a;
            v3 fb = v3_ld(fbt + 3 * i), fp = v3_ld(fpt + 3 * i);
            if (!frozen(sys, r, a >> 1) && P->gamma > 0.0) {
                v3 V = v3_ld(S->V + 3 * i), u = v3_ld(S->u + 3 * i);
                v3 w = v3_mul(v3_ld(S->L + 3 * i), 1.0 / I);
                v3 vb = v3_add(V, v3_cross(w, v3_mul(u, -db)));
                v3 vp = v3_add(V, v3_cross(w, v3_mul(u, dp)));
                double xi[6];
                orc_noise(P->seed, P->noise_kind, (uint64_t)S->step, i, 0, xi);
                v3 nb = {xi[0], xi[1], xi[2]}, np = {xi[3], xi[4], xi[5]};
                fb = v3_add(fb, v3_add(v3_mul(vb, -P->gamma), v3_mul(nb, amp)));
                fp = v3_add(fp, v3_add(v3_mul(vp, -P->gamma), v3_mul(np, amp)));
            }
            v3_st(S->fb + 3 * i, fb);
            v3_st(S->fp + 3 * i, fp);
        }
    }
    free(bead);
    free(patch);
    free(fbt);
    free(fpt);
    return st;
}

/* Half kick of the body from its site forces: F = f_b + f_p and the torque
 * about R, tau = (r_b - R) x f_b + (r_p - R) x f_p = u x (dp f_p - db f_b). */
static void half_kick(const orc_params *P, orc_state *S, int64_t i)
{
    double M = P->m_bead + P->m_patch;
    double db = P->ell * P->m_patch / M, dp = P->ell * P->m_bead / M;
    v3 fb = v3_ld(S->fb + 3 * i), fp = v3_ld(S->fp + 3 * i), u = v3_ld(S->u + 3 * i);
    v3 F = v3_add(fb, fp);
    v3 tau = v3_cross(u, v3_sub(v3_mul(fp, dp), v3_mul(fb, db)));
    v3_st(S->V + 3 * i, v3_add(v3_ld(S->V + 3 * i), v3_mul(F, 0.5 * P->dt / M)));
    v3_st(S->L + 3 * i, v3_add(v3_ld(S->L + 3 * i), v3_mul(tau, 0.5 * P->dt)));
}

/* Drift: R += dt V; the axis of a free linear rotor turns about omega = L/I
 * by |omega| dt (Rodrigues' formula); u is renormalised and the component of L
 * along the new axis (carrying no inertia) is removed. */
static void drift(const orc_params *P, orc_state *S, int64_t i)
{
    double M = P->m_bead + P->m_patch;
    double I = P->m_bead * P->m_patch / M * P->ell * P->ell;
    v3 R = v3_ld(S->R + 3 * i), V = v3_ld(S->V + 3 * i), u = v3_ld(S->u + 3 * i);
    v3 L = v3_ld(S->L + 3 * i);
    v3_st(S->R + 3 * i, v3_add(R, v3_mul(V, P->dt)));
    v3 w = v3_mul(L, 1.0 / I);
    double wl = v3_len(w);
    if (wl > 0.0) {
        double th = wl * P->dt;
        v3 k = v3_mul(w, 1.0 / wl);
        double c = cos(th), s = sin(th);
        u = v3_add(v3_add(v3_mul(u, c), v3_mul(v3_cross(k, u), s)),
                   v3_mul(k, v3_dot(k, u) * (1.0 - c)));
    }
    u = v3_mul(u, 1.0 / v3_len(u));
    L = v3_sub(L, v3_mul(u, v3_dot(L, u)));
    v3_st(S->u + 3 * i, u);
    v3_st(S->L + 3 * i, L);
}

/* Appendix A: NVT velocity-Verlet with the Langevin forces evaluated at the
 * half-step velocities.  One step k -> k+1:
 *   kick (dt/2) with the forces of step k, drift, forces of step k+1 (noise
 *   keyed by step k+1), kick (dt/2).
 * Anchored bodies (first base pair of a tethered replica) do not move.
 * Returns ORC_OK or the first error; *err_step and *err_id locate it. */
int orc_step(const orc_params *P, const orc_system *sys, orc_state *S, int64_t nsteps,
             int use_cells, int64_t *err_step, int64_t *err_id)
{
    int64_t N = S->n_nt;
    if (err_step) *err_step = -1;
    if (!S->has_f) {
        int st = total_forces(P, sys, S, use_cells, err_id);
        if (st) { if (err_step) *err_step = S->step; return st; }
        S->has_f = 1;
    }
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int r = 0; r < sys->n_rep; ++r) {
            int64_t off = rep_offset(sys, r);
            for (int64_t a = 0; a < 2 * (int64_t)sys->n_bp[r]; ++a) {
                int64_t i = off + a;
                if (frozen(sys, r, a >> 1)) {
                    memset(S->V + 3 * i, 0, 3 * sizeof(double));
                    memset(S->L + 3 * i, 0, 3 * sizeof(double));
                    continue;
                }
                half_kick(P, S, i);
                drift(P, S, i);
            }
        }
        S->step += 1;
        int st = total_forces(P, sys, S, use_cells, err_id);
        for (int64_t i = 0; i < 3 * N; ++i)
            if (!isfinite(S->R[i]) || !isfinite(S->u[i])) {
                if (st == ORC_OK) { st = ORC_ENAN; if (err_id) *err_id = i / 3; }
                break;
            }
        if (st) { if (err_step) *err_step = S->step; return st; }
        for (int r = 0; r < sys->n_rep; ++r) {
            int64_t off = rep_offset(sys, r);
            for (int64_t a = 0; a < 2 * (int64_t)sys->n_bp[r]; ++a)
                if (!frozen(sys, r, a >> 1)) half_kick(P, S, off + a);
        }
    }
    return ORC_OK;
}

/* Initial velocities: Maxwell-Boltzmann at temperature kT from noise stream 1
 * (step 0): V ~ N(0, kT/M) per component; L ~ N(0, I kT) per component with
 * the part along u removed (a linear rotor has two rotational degrees of
 * freedom).  Anchored bodies get V = L = 0.  Clears the stored forces. */
void orc_thermalize(const orc_params *P, const orc_system *sys, orc_state *S, double kT,
                    uint64_t seed)
{
    double M = P->m_bead + P->m_patch;
    double I = P->m_bead * P->m_patch / M * P->ell * P->ell;
    for (int r = 0; r < sys->n_rep; ++r) {
        int64_t off = rep_offset(sys, r);
        for (int64_t a = 0; a < 2 * (int64_t)sys->n_bp[r]; ++a) {
            int64_t i = off + a;
            double xi[6];
            orc_noise(seed, 0, 0, i, 1, xi);
            v3 V = {xi[0], xi[1], xi[2]}, L = {xi[3], xi[4], xi[5]};
            V = v3_mul(V, sqrt(kT / M));
            L = v3_mul(L, sqrt(I * kT));
            v3 u = v3_ld(S->u + 3 * i);
            L = v3_sub(L, v3_mul(u, v3_dot(L, u)));
            if (frozen(sys, r, a >> 1)) { V = v3_mul(V, 0.0); L = v3_mul(L, 0.0); }
            v3_st(S->V + 3 * i, V);
            v3_st(S->L + 3 * i, L);
        }
    }
    S->has_f = 0;
}

/* Kinetic energies per replica: translational sum M V^2/2 and rotational
 * sum L^2/(2I). */
void orc_kinetic(const orc_params *P, const orc_system *sys, const orc_state *S, double *ke_t,
                 double *ke_r)
{
    double M = P->m_bead + P->m_patch;
    double I = P->m_bead * P->m_patch / M * P->ell * P->ell;
    for (int r = 0; r < sys->n_rep; ++r) {
        int64_t off = rep_offset(sys, r);
        double kt = 0.0, kr = 0.0;
        for (int64_t a = 0; a < 2 * (int64_t)sys->n_bp[r]; ++a) {
            int64_t i = off + a;
            kt += 0.5 * M * v3_dot(v3_ld(S->V + 3 * i), v3_ld(S->V + 3 * i));
            kr += 0.5 * v3_dot(v3_ld(S->L + 3 * i), v3_ld(S->L + 3 * i)) / I;
        }
        ke_t[r] = kt;
        ke_r[r] = kr;
    }
}

/* Bubble statistics of Sec. 5 for one open mask: fraction of open base pairs
 * and the histogram of maximal open-run lengths (hist[k] counts runs of
 * length k, k < nhist; longer runs land in hist[nhist-1]).  On a ring
 * (ring != 0) runs are cyclic: a run through bp nbp-1 and bp 0 counts once,
 * and a ring with every base pair open is one run of length nbp. */
void orc_bubbles(const uint8_t *open, int64_t nbp, int ring, double *frac, int64_t *hist, int nhist)
{
    int64_t nopen = 0;
    for (int k = 0; k < nhist; ++k) hist[k] = 0;
    int64_t c = 0; /* runs are read starting after the closed bp c */
    if (ring) {
        while (c < nbp && open[c]) ++c;
        if (c == nbp) {
            if (nbp) hist[nbp < nhist ? nbp : nhist - 1] += 1;
            *frac = nbp ? 1.0 : 0.0;
            return;
        }
    }
    int64_t k = 0;
    while (k < nbp) {
        int64_t n = ring ? (c + k) % nbp : k;
        if (!open[n]) { ++k; continue; }
        int64_t e = k;
        while (e < nbp && open[ring ? (c + e) % nbp : e]) ++e;
        int64_t len = e - k;
        nopen += len;
        hist[len < nhist ? len : nhist - 1] += 1;
        k = e;
    }
    *frac = nbp ? (double)nopen / (double)nbp : 0.0;
}

int orc_nterm(void) { return NTERM; }
size_t orc_sizeof_params(void) { return sizeof(orc_params); }
size_t orc_sizeof_system(void) { return sizeof(orc_system); }
size_t orc_sizeof_state(void) { return sizeof(orc_state); }
