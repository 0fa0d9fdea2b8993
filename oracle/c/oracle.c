/*
 * FP64 CPU oracle for the Gaussian bilateral filter and its polynomial
 * (Gauss-Chebyshev / Gauss-polynomial) approximation.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark. It shares no code with the GPU library.
 *
 * Plain loops, OpenMP over output rows. Notation follows the paper
 * (Ghosh & Chaudhury 2016):
 *   image f on a rectangle, extended outside it by symmetry (Section I;
 *   read as the half-sample mirror, period 2M);
 *   spatial kernel g_s(j) = exp(-|j|^2 / 2 sigma_s^2) on the square
 *   Omega = [-W, W]^2, W = 3 sigma_s rounded up (Section I);
 *   range kernel g_r(t) = exp(-t^2 / 2 sigma_r^2).
 *
 * All routines compute the output on a region [r0, r1) x [c0, c1) of the
 * image; pixels outside the image are read through the symmetric extension.
 * Return 0 on success, -1 on invalid arguments, -2 when memory runs out.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static long mirror(long i, long M)
{
    long p = i % (2 * M);
    if (p < 0) p += 2 * M;
    return p >= M ? 2 * M - 1 - p : p;
}

static int radius_of(double sigma_s)
{
    return (int)ceil(3.0 * sigma_s - 1e-12);
}

static int check_region(int H, int Wd, int r0, int r1, int c0, int c1)
{
    return H >= 1 && Wd >= 1 && 0 <= r0 && r0 <= r1 && r1 <= H && 0 <= c0 && c0 <= c1 && c1 <= Wd;
}

/* Eq. (1): brute force over Omega. */
int oracle_direct_bf(const double *f, int H, int Wd, long ld, double sigma_s, double sigma_r,
                     int r0, int r1, int c0, int c1, double *out, long ldo)
{
    if (!f || !out || !(sigma_s > 0) || !(sigma_r > 0) || !check_region(H, Wd, r0, r1, c0, c1))
        return -1;
    const int W = radius_of(sigma_s);
    const double as = 1.0 / (2.0 * sigma_s * sigma_s);
    const double ar = 1.0 / (2.0 * sigma_r * sigma_r);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = r0; r < r1; ++r) {
        for (int c = c0; c < c1; ++c) {
            const double fi = f[(long)r * ld + c];
            double num = 0.0, den = 0.0;
            for (int j1 = -W; j1 <= W; ++j1) {
                const long rr = mirror(r - j1, H);
                for (int j2 = -W; j2 <= W; ++j2) {
                    const long cc = mirror(c - j2, Wd);
                    const double t = f[rr * ld + cc];
                    const double d = t - fi;
                    const double w = exp(-(double)(j1 * j1 + j2 * j2) * as) * exp(-d * d * ar);
                    num += w * t;
                    den += w;
                }
            }
            out[(long)(r - r0) * ldo + (c - c0)] = num / den;
        }
    }
    return 0;
}

/*
 * The fast algorithm of Section II for exp(x) ~ sum_{n=0}^{N} c_n x^n, on the
 * image centred at t_c (eq. 17), centring undone at the end (Section III-B):
 *   G_n = (g/sigma_r)^n,  F_n = exp(-g^2/2 sigma_r^2) G_n          (eq. 6)
 *   F_bar_n = sum_{j in Omega} g_s(j) F_n(i - j),  n = 0..N+1         (eq. 7)
 *   P = sigma_r sum_n c_n G_n F_bar_{n+1},  Q = sum_n c_n G_n F_bar_n (eq. 8, 9)
 *   out = P / Q + t_c                                                  (eq. 10)
 * Eq. (7) is evaluated through separability of g_s on the square Omega: a
 * 1-D pass along rows over the region grown by W rows, then along columns.
 * P_out and Q_out (optional, may be NULL) receive P and Q on the region.
 */
int oracle_polynomial_filter(const double *f, int H, int Wd, long ld, double sigma_s, double sigma_r,
                             int N, const double *c, double t_c,
                             int r0, int r1, int c0, int c1,
                             double *out, long ldo, double *P_out, double *Q_out)
{
    if (!f || !out || !c || N < 0 || !(sigma_s > 0) || !(sigma_r > 0) ||
        !check_region(H, Wd, r0, r1, c0, c1))
        return -1;
    const int W = radius_of(sigma_s);
    const long h = r1 - r0, w = c1 - c0;
    const long he = h + 2L * W, we = w + 2L * W;   /* region grown by W */
    if (h == 0 || w == 0) return 0;

    double *taps = malloc(sizeof(double) * (2 * W + 1));
    double *u = malloc(sizeof(double) * he * we);     /* g / sigma_r on the grown region */
    double *Fn = malloc(sizeof(double) * he * we);    /* F_n on the grown region         */
    double *tmp = malloc(sizeof(double) * he * w);    /* row-filtered F_n                */
    double *Fb = malloc(sizeof(double) * h * w);      /* F_bar_n on the region           */
    double *Gc = malloc(sizeof(double) * h * w);      /* G_n at the region's pixels      */
    double *P = malloc(sizeof(double) * h * w);
    double *Q = malloc(sizeof(double) * h * w);
    if (!taps || !u || !Fn || !tmp || !Fb || !Gc || !P || !Q) {
        free(taps); free(u); free(Fn); free(tmp); free(Fb); free(Gc); free(P); free(Q);
        return -2;
    }
    for (int k = -W; k <= W; ++k)
        taps[k + W] = exp(-(double)(k * k) / (2.0 * sigma_s * sigma_s));

    #pragma omp parallel for
    for (long a = 0; a < he; ++a) {
        const long rr = mirror(r0 - W + a, H);
        for (long b = 0; b < we; ++b) {
            const long cc = mirror(c0 - W + b, Wd);
            const double g = f[rr * ld + cc] - t_c;                        /* eq. (17) */
            u[a * we + b] = g / sigma_r;
            Fn[a * we + b] = exp(-g * g / (2.0 * sigma_r * sigma_r));      /* F_0 */
        }
    }
    #pragma omp parallel for
    for (long a = 0; a < h; ++a)
        for (long b = 0; b < w; ++b) {
            Gc[a * w + b] = 1.0;                                           /* G_0 */
            P[a * w + b] = 0.0;
            Q[a * w + b] = 0.0;
        }

    for (int n = 0; n <= N + 1; ++n) {
        if (n > 0) {                                                       /* F_n = F_{n-1} g/sigma_r */
            #pragma omp parallel for
            for (long a = 0; a < he; ++a)
                for (long b = 0; b < we; ++b)
                    Fn[a * we + b] *= u[a * we + b];
        }
        /* eq. (7), rows then columns */
        #pragma omp parallel for
        for (long a = 0; a < he; ++a)
            for (long b = 0; b < w; ++b) {
                double s = 0.0;
                for (int k = -W; k <= W; ++k)
                    s += taps[k + W] * Fn[a * we + (b + W - k)];
                tmp[a * w + b] = s;
            }
        #pragma omp parallel for
        for (long a = 0; a < h; ++a)
            for (long b = 0; b < w; ++b) {
                double s = 0.0;
                for (int k = -W; k <= W; ++k)
                    s += taps[k + W] * tmp[(a + W - k) * w + b];
                Fb[a * w + b] = s;
            }
        /* eq. (8) takes F_bar_{n} with c_{n-1} G_{n-1}; eq. (9) takes F_bar_n with c_n G_n */
        #pragma omp parallel for
        for (long a = 0; a < h; ++a)
            for (long b = 0; b < w; ++b) {
                const long i = a * w + b;
                if (n >= 1) P[i] += sigma_r * c[n - 1] * Gc[i] * Fb[i];
                if (n <= N) {
                    if (n >= 1) Gc[i] *= u[(a + W) * we + (b + W)];
                    Q[i] += c[n] * Gc[i] * Fb[i];
                }
            }
    }
    for (long a = 0; a < h; ++a)
        for (long b = 0; b < w; ++b) {
            const long i = a * w + b;
            out[a * ldo + b] = P[i] / Q[i] + t_c;                           /* eq. (10) */
            if (P_out) P_out[a * w + b] = P[i];
            if (Q_out) Q_out[a * w + b] = Q[i];
        }
    free(taps); free(u); free(Fn); free(tmp); free(Fb); free(Gc); free(P); free(Q);
    return 0;
}
