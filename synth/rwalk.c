/*
 * rwalk.c -- input generator: the axis of a long duplex laid out as a
 * persistent random walk in a periodic cube with self-avoidance.  Part of the
 * seeded synthetic-input module; it holds no force-field or integrator code.
 *
 * The axis is a chain of seg_bp-point segments spaced `rise` apart.  From one
 * segment to the next the direction turns by arccos(1 - 0.362 xi), xi ~ U(0,1),
 * about a uniformly random axis perpendicular to it; within a segment the
 * tangent turns uniformly, so the axis has no kinks.  A normal vector e1 is
 * carried along by the same rotations (parallel transport).
 *
 * Self-avoidance uses an occupancy grid of cells of edge >= excl/2 that
 * records the first segment to enter each cell.  A candidate segment is
 * rejected when one of its points (past the first three) has, within two
 * cells, a cell first entered more than `window` segments earlier.  After
 * max_tries/2 rejections the turn angle is drawn uniformly in [0, 90 deg];
 * after max_tries the walk backs up four segments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_state;
static uint64_t splitmix64(void)
{
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double uni(void) { return (double)(splitmix64() >> 11) * 0x1p-53; }

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize(double *v)
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}
/* rotate v about unit axis a by angle th (Rodrigues) */
static void rot(const double *v, const double *a, double th, double *o)
{
    double c = cos(th), s = sin(th), ax[3];
    cross(a, v, ax);
    double ad = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    for (int k = 0; k < 3; ++k) o[k] = v[k] * c + ax[k] * s + a[k] * ad * (1.0 - c);
}
/* two unit vectors perpendicular to unit t */
static void perp(const double *t, double *p1, double *p2)
{
    double a[3] = {1.0, 0.0, 0.0};
    if (fabs(t[0]) >= 0.9) { a[0] = 0.0; a[1] = 1.0; }
    double d = a[0] * t[0] + a[1] * t[1] + a[2] * t[2];
    for (int k = 0; k < 3; ++k) p1[k] = a[k] - t[k] * d;
    normalize(p1);
    cross(t, p1, p2);
}

/* Returns 0 on success, -1 when the walk cannot be placed.  Outputs hold
 * n_seg * seg_bp points each ([.., 3]). */
int rw_generate(int64_t n_seg, int seg_bp, double L, double rise, double excl, int window, int max_tries,
                uint64_t seed, const double *d0, const double *pos0, double *axis, double *tang, double *e1out,
                int64_t *n_backups)
{
    sm_state = seed;
    int use_grid = excl > 0.0;
    int64_t ng = use_grid ? (int64_t)floor(L / (excl / 2.0)) : 1;
    if (ng < 5) ng = 5;
    if (ng > 2048) ng = 2048;
    double cw = L / (double)ng;
    int32_t *occ = NULL;
    int64_t *first = NULL, *first_off = NULL; /* per segment: cells it entered first */
    if (use_grid) {
        occ = (int32_t *)malloc(sizeof(int32_t) * ng * ng * ng);
        if (!occ) return -1;
        for (int64_t q = 0; q < ng * ng * ng; ++q) occ[q] = -1;
    }
    first = (int64_t *)malloc(sizeof(int64_t) * (n_seg * seg_bp + 1));
    first_off = (int64_t *)malloc(sizeof(int64_t) * (n_seg + 1));
    double *hist = (double *)malloc(sizeof(double) * 9 * (n_seg + 1));
    double *pts = (double *)malloc(sizeof(double) * 3 * seg_bp);
    double *tt = (double *)malloc(sizeof(double) * 3 * seg_bp);
    if (!first || !first_off || !hist || !pts || !tt) { free(occ); free(first); free(first_off); free(hist); free(pts); free(tt); return -1; }
    first_off[0] = 0;

    double pos[3] = {pos0[0], pos0[1], pos0[2]}, d[3] = {d0[0], d0[1], d0[2]}, e1[3], p2[3];
    normalize(d);
    perp(d, e1, p2);
    int64_t k = 0, backups = 0;
    while (k < n_seg) {
        memcpy(hist + 9 * k, pos, sizeof pos);
        memcpy(hist + 9 * k + 3, d, sizeof d);
        memcpy(hist + 9 * k + 6, e1, sizeof e1);
        double q1[3], q2[3];
        perp(d, q1, q2);
        int ok = 0;
        double th = 0.0, a[3] = {0, 0, 0};
        for (int attempt = 0; attempt < max_tries && !ok; ++attempt) {
            th = attempt < max_tries / 2 ? acos(1.0 - 0.362 * uni()) : 0.5 * M_PI * uni();
            double phi = 2.0 * M_PI * uni();
            for (int m = 0; m < 3; ++m) a[m] = cos(phi) * q1[m] + sin(phi) * q2[m];
            double axd[3];
            cross(a, d, axd);
            double acc[3] = {0, 0, 0};
            for (int j = 0; j < seg_bp; ++j) {
                double ang = j * (th / seg_bp), c = cos(ang), s = sin(ang);
                for (int m = 0; m < 3; ++m) {
                    tt[3 * j + m] = c * d[m] + s * axd[m];
                    pts[3 * j + m] = pos[m] + rise * acc[m];
                }
                for (int m = 0; m < 3; ++m) acc[m] += tt[3 * j + m];
            }
            ok = 1;
            if (use_grid) {
                for (int j = 3; j < seg_bp && ok; ++j) {
                    int64_t c[3];
                    for (int m = 0; m < 3; ++m) {
                        double x = fmod(pts[3 * j + m], L);
                        if (x < 0) x += L;
                        c[m] = (int64_t)floor(x / cw) % ng;
                    }
                    for (int dz = -2; dz <= 2 && ok; ++dz)
                        for (int dy = -2; dy <= 2 && ok; ++dy)
                            for (int dx = -2; dx <= 2 && ok; ++dx) {
                                int64_t x = (c[0] + dx + ng) % ng, y = (c[1] + dy + ng) % ng,
                                        z = (c[2] + dz + ng) % ng;
                                int32_t o = occ[(z * ng + y) * ng + x];
                                if (o >= 0 && o < k - window) ok = 0;
                            }
                }
            }
        }
        if (!ok) {
            int64_t back = k < 4 ? k : 4;
            for (int64_t q = k - 1; q >= k - back; --q)
                for (int64_t f = first_off[q]; f < first_off[q + 1]; ++f) occ[first[f]] = -1;
            k -= back;
            memcpy(pos, hist + 9 * k, sizeof pos);
            memcpy(d, hist + 9 * k + 3, sizeof d);
            memcpy(e1, hist + 9 * k + 6, sizeof e1);
            if (++backups > 50 * n_seg) { free(occ); free(first); free(first_off); free(hist); free(pts); free(tt); return -1; }
            continue;
        }
        /* accept: outputs, occupancy, next frame */
        int64_t nf = first_off[k];
        for (int j = 0; j < seg_bp; ++j) {
            double ang = j * (th / seg_bp), e[3];
            rot(e1, a, ang, e);
            for (int m = 0; m < 3; ++m) {
                axis[3 * (k * seg_bp + j) + m] = pts[3 * j + m];
                tang[3 * (k * seg_bp + j) + m] = tt[3 * j + m];
                e1out[3 * (k * seg_bp + j) + m] = e[m];
            }
            if (use_grid) {
                int64_t c[3];
                for (int m = 0; m < 3; ++m) {
                    double x = fmod(pts[3 * j + m], L);
                    if (x < 0) x += L;
                    c[m] = (int64_t)floor(x / cw) % ng;
                }
                int64_t flat = (c[2] * ng + c[1]) * ng + c[0];
                if (occ[flat] < 0) { occ[flat] = (int32_t)k; first[nf++] = flat; }
            }
        }
        first_off[k + 1] = nf;
        double dn[3], en[3];
        rot(d, a, th, dn);
        rot(e1, a, th, en);
        normalize(dn);
        double pe = en[0] * dn[0] + en[1] * dn[1] + en[2] * dn[2];
        for (int m = 0; m < 3; ++m) en[m] -= pe * dn[m];
        normalize(en);
        for (int m = 0; m < 3; ++m) {
            pos[m] = pts[3 * (seg_bp - 1) + m] + rise * tt[3 * (seg_bp - 1) + m];
            d[m] = dn[m];
            e1[m] = en[m];
        }
        ++k;
    }
    *n_backups = backups;
    free(occ); free(first); free(first_off); free(hist); free(pts); free(tt);
    return 0;
}
