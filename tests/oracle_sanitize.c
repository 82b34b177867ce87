/*
 * Sanitizer driver for the FP64 oracle (test infrastructure): built by the
 * CPU tests with gcc's AddressSanitizer and UndefinedBehaviorSanitizer and
 * without them, it runs every exported oracle function on the configuration
 * in argv[1] and prints one checksum line per call, so that the two builds
 * can be compared bit for bit and any invalid access or undefined operation
 * stops the sanitized run.
 *
 * Input (native byte order, written by the test):
 *   int64 n_rep; int32 n_bp[n_rep]; uint8 circular[n_rep];
 *   uint8 periodic[n_rep][3]; double box[n_rep][6]; double pull[n_rep][3];
 *   double torque[n_rep][3]; uint8 tether[n_rep]; double wall_z[n_rep];
 *   double k2_scale[n_rep]; double k2_bp[sum n_bp];
 *   double bead[N][3]; double patch[N][3]       (N = 2 sum n_bp)
 */
#include "../oracle/dsdna_oracle.c"

#include <stdio.h>

static void *rd(FILE *f, size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p || fread(p, 1, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static double sum(const double *x, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * (double)(1 + (i % 7));
    return s;
}

static orc_params defaults(void)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.K1 = 30.0; p.R0 = 0.6825; p.eps_bb = 1.0; p.sig_bb = 0.4430;
    p.K2 = 6.0; p.r0_hb = 0.0; p.rc_hb = 0.3;
    p.eps = 1.0; p.sig_s = 1.0; p.sig_x = 0.5;
    p.K3 = 50.0; p.d_dih = -144.0 * M_PI / 180.0;
    p.K4 = 30.0; p.lam = 8.0; p.r0_m = 0.34;
    p.K5 = 200.0; p.a0 = M_PI / 2.0;
    p.K6 = 52.0;
    p.ell = 0.5; p.m_bead = 1.0; p.m_patch = 1.0;
    p.gamma = 1.0; p.kT = 1.0; p.dt = 0.005;
    p.seed = 7;
    return p;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t *nr = (int64_t *)rd(f, sizeof(int64_t));
    const int R = (int)*nr;
    int32_t *n_bp = (int32_t *)rd(f, sizeof(int32_t) * R);
    uint8_t *circ = (uint8_t *)rd(f, (size_t)R);
    uint8_t *per = (uint8_t *)rd(f, (size_t)R * 3);
    double *box = (double *)rd(f, sizeof(double) * R * 6);
    double *pull = (double *)rd(f, sizeof(double) * R * 3);
    double *torque = (double *)rd(f, sizeof(double) * R * 3);
    uint8_t *tether = (uint8_t *)rd(f, (size_t)R);
    double *wall = (double *)rd(f, sizeof(double) * R);
    double *k2s = (double *)rd(f, sizeof(double) * R);
    int64_t nbp = 0;
    for (int r = 0; r < R; ++r) nbp += n_bp[r];
    const int64_t N = 2 * nbp;
    double *k2bp = (double *)rd(f, sizeof(double) * nbp);
    double *bead = (double *)rd(f, sizeof(double) * N * 3);
    double *patch = (double *)rd(f, sizeof(double) * N * 3);
    fclose(f);
    free(nr);

    orc_system sys = {R, n_bp, box, per, pull, torque, tether, wall, k2s, circ, k2bp};
    double *fb = (double *)calloc((size_t)NTERM * N * 3, sizeof(double));
    double *fp = (double *)calloc((size_t)NTERM * N * 3, sizeof(double));
    double *E = (double *)calloc((size_t)R * NTERM, sizeof(double));
    uint8_t *open = (uint8_t *)calloc((size_t)nbp, 1);
    int64_t err = -1;

    /* forces under every reading switch, all pairs and cell search */
    for (int variant = 0; variant < 6; ++variant) {
        orc_params P = defaults();
        P.ssdna_rule = variant >= 1;
        P.dihedral_damping = variant == 2 || variant == 5;
        P.planarity_both = variant == 3 || variant == 5;
        P.fene_clamp = variant == 4;
        P.hb_depth_convention = variant == 4;
        for (int cells = 0; cells < 2; ++cells)
            for (int split = 0; split < 2; ++split) {
                int st = orc_forces(&P, &sys, bead, patch, cells, split, fb, fp, E, open, &err);
                int64_t n = (split ? NTERM : 1) * N * 3;
                int64_t no = 0;
                for (int64_t k = 0; k < nbp; ++k) no += open[k];
                printf("forces v%d c%d s%d st=%d err=%lld %.17g %.17g %.17g open=%lld\n", variant, cells, split, st,
                       (long long)err, sum(fb, n), sum(fp, n), sum(E, (int64_t)R * NTERM), (long long)no);
            }
    }

    /* bodies <-> sites */
    orc_params P = defaults();
    P.ssdna_rule = 1;
    double *Rb = (double *)malloc(sizeof(double) * N * 3), *u = (double *)malloc(sizeof(double) * N * 3);
    double *V = (double *)calloc((size_t)N * 3, sizeof(double)), *L = (double *)calloc((size_t)N * 3, sizeof(double));
    double *sb = (double *)malloc(sizeof(double) * N * 3), *sp = (double *)malloc(sizeof(double) * N * 3);
    orc_bodies_from_sites(&P, N, bead, patch, Rb, u);
    orc_sites_from_bodies(&P, N, Rb, u, sb, sp);
    printf("bodies %.17g %.17g %.17g\n", sum(Rb, N * 3), sum(u, N * 3), sum(sb, N * 3) + sum(sp, N * 3));

    /* thermalize, step (cell search), kinetic energy */
    double *tfb = (double *)calloc((size_t)N * 3, sizeof(double)), *tfp = (double *)calloc((size_t)N * 3, sizeof(double));
    orc_state S = {N, Rb, u, V, L, tfb, tfp, 0, 0, 0};
    orc_thermalize(&P, &sys, &S, 1.0, 11);
    int64_t es = -1, ei = -1;
    int st = orc_step(&P, &sys, &S, 25, 1, &es, &ei);
    double *kt = (double *)calloc((size_t)R, sizeof(double)), *kr = (double *)calloc((size_t)R, sizeof(double));
    orc_kinetic(&P, &sys, &S, kt, kr);
    printf("step st=%d es=%lld ei=%lld %.17g %.17g %.17g %.17g\n", st, (long long)es, (long long)ei,
           sum(Rb, N * 3), sum(V, N * 3), sum(kt, R), sum(kr, R));

    /* neighbour pairs of every replica, both searches */
    int64_t cap = 1 << 16;
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * 2 * cap);
    for (int r = 0; r < R; ++r)
        for (int cells = 0; cells < 2; ++cells) {
            int64_t np = orc_wca_pairs(&P, &sys, bead, r, cells, pairs, cap);
            long long s = 0;
            for (int64_t k = 0; k < (np < cap ? np : cap); ++k) s += pairs[2 * k] * 31 + pairs[2 * k + 1];
            printf("pairs r%d c%d n=%lld %lld\n", r, cells, (long long)np, s);
        }

    /* bubbles of the open flags of each replica, linear and cyclic */
    orc_forces(&P, &sys, bead, patch, 1, 0, fb, fp, E, open, &err);
    int64_t base = 0;
    for (int r = 0; r < R; ++r) {
        for (int ring = 0; ring < 2; ++ring) {
            double frac = 0.0;
            int64_t hist[9] = {0};
            orc_bubbles(open + base, n_bp[r], ring, &frac, hist, 9);
            long long h = 0;
            for (int k = 0; k < 9; ++k) h = h * 7 + hist[k];
            printf("bubbles r%d ring%d %.17g %lld\n", r, ring, frac, h);
        }
        base += n_bp[r];
    }

    /* noise and the counter-based generators */
    double xi[6];
    for (int kind = 0; kind < 2; ++kind) {
        double s = 0.0;
        for (int64_t id = 0; id < 64; ++id) {
            orc_noise(3, kind, 12345 + id, id * 977, (int)(id & 1), xi);
            s += sum(xi, 6);
        }
        printf("noise k%d %.17g\n", kind, s);
    }
    uint32_t c32[4] = {1, 2, 3, 4}, k32[2] = {5, 6}, o32[4];
    orc_philox4x32(c32, k32, o32);
    uint64_t c64[4] = {1, 2, 3, 4}, k64[2] = {5, 6}, o64[4];
    orc_philox4x64(c64, k64, o64);
    printf("philox %u %u %u %u %llu %llu\n", o32[0], o32[1], o32[2], o32[3], (unsigned long long)o64[0],
           (unsigned long long)o64[3]);
    printf("sizes %d %zu %zu %zu\n", orc_nterm(), orc_sizeof_params(), orc_sizeof_system(), orc_sizeof_state());

    free(n_bp); free(circ); free(per); free(box); free(pull); free(torque); free(tether); free(wall); free(k2s);
    free(k2bp); free(bead); free(patch); free(fb); free(fp); free(E); free(open); free(Rb); free(u); free(V);
    free(L); free(sb); free(sp); free(tfb); free(tfp); free(kt); free(kr); free(pairs);
    return 0;
}
