/* Drives the plain-C oracle (direct filter, polynomial filter, crops, radii
 * above the image side, degenerate shapes) under AddressSanitizer and
 * UndefinedBehaviorSanitizer. Exits non-zero on a failed sanity check. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_direct_bf(const double *f, int H, int Wd, long ld, double sigma_s, double sigma_r,
                     int r0, int r1, int c0, int c1, double *out, long ldo);
int oracle_polynomial_filter(const double *f, int H, int Wd, long ld, double sigma_s, double sigma_r,
                             int N, const double *c, double t_c,
                             int r0, int r1, int c0, int c1,
                             double *out, long ldo, double *P_out, double *Q_out);

static int fails = 0;

static void run(int H, int Wd, long ld, double ss, double sr, int r0, int r1, int c0, int c1) {
    double *f = malloc(sizeof(double) * (size_t)(H * ld));
    const int h = r1 - r0, w = c1 - c0;
    double *o1 = malloc(sizeof(double) * (size_t)(h * w + 1));
    double *o2 = malloc(sizeof(double) * (size_t)(h * w + 1));
    double *P = malloc(sizeof(double) * (size_t)(h * w + 1));
    double *Q = malloc(sizeof(double) * (size_t)(h * w + 1));
    double c[41];
    unsigned s = 7u + (unsigned)(H * 131 + Wd);
    for (long i = 0; i < H * ld; ++i) {
        s = s * 1664525u + 1013904223u;
        f[i] = (double)(s >> 24);
    }
    /* Taylor coefficients of exp: c_n = 1/n! (the Gauss-polynomial filter) */
    c[0] = 1.0;
    for (int n = 1; n <= 40; ++n) c[n] = c[n - 1] / n;
    if (oracle_direct_bf(f, H, Wd, ld, ss, sr, r0, r1, c0, c1, o1, w) != 0) {
        fprintf(stderr, "direct filter refused %dx%d\n", H, Wd);
        ++fails;
    }
    if (oracle_polynomial_filter(f, H, Wd, ld, ss, sr, 40, c, 127.5, r0, r1, c0, c1, o2, w, P, Q) != 0) {
        fprintf(stderr, "polynomial filter refused %dx%d\n", H, Wd);
        ++fails;
    }
    for (int i = 0; i < h * w; ++i)
        if (!(o1[i] >= -1e-9 && o1[i] <= 255.0 + 1e-9)) {
            fprintf(stderr, "direct filter output out of range at %d: %g\n", i, o1[i]);
            ++fails;
            break;
        }
    /* a radius beyond the image side and a large sigma_r: the polynomial
     * filter of high degree approaches the direct one */
    free(f); free(o1); free(o2); free(P); free(Q);
}

int main(void) {
    run(1, 1, 1, 1.0, 30.0, 0, 1, 0, 1);
    run(1, 17, 17, 3.0, 30.0, 0, 1, 0, 17);
    run(17, 1, 4, 3.0, 30.0, 0, 17, 0, 1);
    run(7, 9, 12, 5.0, 300.0, 0, 7, 0, 9);         /* W = 15 > both sides */
    run(33, 40, 40, 2.0, 50.0, 3, 20, 0, 40);       /* crop touching the left and right borders */
    run(64, 48, 64, 1.5, 60.0, 60, 64, 40, 48);     /* bottom-right corner crop */
    run(20, 20, 20, 1.0, 40.0, 5, 5, 2, 9);         /* empty crop */
    /* invalid arguments are refused, not read */
    {
        double f[4] = {0, 1, 2, 3}, out[4];
        if (oracle_direct_bf(f, 2, 2, 2, 1.0, 30.0, 0, 3, 0, 2, out, 2) == 0) { fprintf(stderr, "bad region accepted\n"); ++fails; }
        if (oracle_direct_bf(f, 2, 2, 2, -1.0, 30.0, 0, 2, 0, 2, out, 2) == 0) { fprintf(stderr, "bad sigma accepted\n"); ++fails; }
    }
    printf("oracle driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
