/*
 * A plain C client of the library's C ABI (include/dsdna.h): one ideal 24 bp
 * duplex (Sec. 2 geometry: patches on the axis 0.34 apart, beads 0.5 off it
 * at 36 degrees per base pair, the strands opposite), thermalised and
 * stepped with FP64 forces.  Prints the sites it started from and the body
 * positions after the steps, so a test can repeat the run through the Python
 * binding and compare.  Usage: c_abi_demo [steps]
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "dsdna.h"

#define CHECK(call)                                                                      \
    do {                                                                                 \
        dsdna_status st_ = (call);                                                       \
        if (st_ != DSDNA_OK) {                                                           \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_,                     \
                    ctx ? dsdna_last_error(ctx) : "no context");                         \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

int main(int argc, char **argv)
{
    const int32_t n_bp = 24;
    const int n_nt = 2 * n_bp;
    const long steps = argc > 1 ? atol(argv[1]) : 10;
    dsdna_ctx *ctx = NULL;
    dsdna_params prm;
    CHECK(dsdna_default_params(&prm));
    prm.seed = 7;
    prm.force_fp64 = 1;
    CHECK(dsdna_create(&ctx, &prm, 0, NULL));
    CHECK(dsdna_set_topology(ctx, 1, &n_bp));

    double *bead = malloc(sizeof(double) * 3 * n_nt), *patch = malloc(sizeof(double) * 3 * n_nt);
    double *R = malloc(sizeof(double) * 3 * n_nt);
    if (!bead || !patch || !R) return 1;
    const double pi = 3.14159265358979323846;
    for (int n = 0; n < n_bp; ++n)
        for (int s = 0; s < 2; ++s) {
            const int i = 2 * n + s;
            const double ang = (36.0 * n + 180.0 * s) * pi / 180.0;
            bead[3 * i] = 0.5 * cos(ang);
            bead[3 * i + 1] = 0.5 * sin(ang);
            bead[3 * i + 2] = 0.34 * n;
            patch[3 * i] = 0.0;
            patch[3 * i + 1] = 0.0;
            patch[3 * i + 2] = 0.34 * n;
        }
    CHECK(dsdna_set_sites(ctx, bead, patch));
    CHECK(dsdna_thermalize(ctx, 1.0, 7));
    CHECK(dsdna_step(ctx, steps));
    int64_t k = -1;
    CHECK(dsdna_get_state(ctx, R, NULL, NULL, NULL, &k));
    printf("step %lld\n", (long long)k);
    for (int i = 0; i < n_nt; ++i)
        printf("site %.17g %.17g %.17g %.17g %.17g %.17g\n", bead[3 * i], bead[3 * i + 1], bead[3 * i + 2],
               patch[3 * i], patch[3 * i + 1], patch[3 * i + 2]);
    for (int i = 0; i < n_nt; ++i) printf("R %.17g %.17g %.17g\n", R[3 * i], R[3 * i + 1], R[3 * i + 2]);
    CHECK(dsdna_destroy(ctx));
    ctx = NULL;
    free(bead);
    free(patch);
    free(R);
    return 0;
}
