/*
 * Drives every entry point of the C oracle on small inputs so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer sees all of its code
 * paths: transforms of every line length class (powers of two, factors of
 * three, other lengths), both start rules, linear and nonlinear runs, the 2/3
 * truncation, a blow-up, the complex-field run, the per-mode first step, and
 * rejected arguments.  Test infrastructure: built and run by
 * tests/test_oracle_sanitizers.py, never part of the library.
 *
 * Exit status 0 when every call returns what it should; a sanitizer report
 * aborts the run with its own non-zero status.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int kgo_num_threads(void);
int kgo_fft1d(int n, double *data, int sign);
int kgo_fft3d_axis(int nx, int ny, int nz, double *data, int axis, int sign);
int kgo_fft3d(int nx, int ny, int nz, double *data, int sign);
int kgo_run(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt, int linear_only,
            int dealias, double threshold, int mode, const double *u0, const double *aux,
            int nsteps, double *u_out, double *uprev_out, double *energy, double *maxu,
            double *q4, int *blowup_step, double *loop_seconds);
int kgo_state(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt, int linear_only,
              int dealias, int mode, const double *u0, const double *aux, int nsteps,
              double *v_prev, double *v_cur);
int kgo_first_step_modes(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
                         int linear_only, const double *u0, int nmodes, const int *modes,
                         double *v0_out, double *v1_out);
int kgo_run_c(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt, int linear_only,
              int dealias, double threshold, int mode, const double *u0, const double *aux,
              int nsteps, double *u_out, double *uprev_out, double *energy, double *maxu,
              double *q4, int *blowup_step);

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

/* deterministic values in [-1, 1) */
static double rnd(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 8388608.0 - 1.0;
}

static double *field(int n, double amp, unsigned seed)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)n * n * n);
    const double L = 8.0 * M_PI, h = L / n;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const double X = -L / 2 + x * h, Y = -L / 2 + y * h, Z = -L / 2 + z * h;
                u[((size_t)z * n + y) * n + x] =
                    amp * exp(-(X * X + Y * Y + Z * Z)) + 1e-3 * rnd(&seed);
            }
    return u;
}

static void transforms(void)
{
    static const int lens[] = {1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 18, 24, 30, 48, 64, 96, 128};
    unsigned s = 7;
    for (size_t i = 0; i < sizeof lens / sizeof lens[0]; ++i) {
        const int n = lens[i];
        double *a = (double *)malloc(sizeof(double) * 2 * n), *b = (double *)malloc(sizeof(double) * 2 * n);
        for (int j = 0; j < 2 * n; ++j) a[j] = b[j] = rnd(&s);
        expect(kgo_fft1d(n, a, -1) == 0 && kgo_fft1d(n, a, 1) == 0, "fft1d");
        double err = 0;
        for (int j = 0; j < 2 * n; ++j) err = fmax(err, fabs(a[j] / n - b[j]));
        expect(err < 1e-12, "fft1d round trip");
        free(a);
        free(b);
    }
    const int nx = 12, ny = 6, nz = 10;
    const size_t m = (size_t)nx * ny * nz;
    double *a = (double *)malloc(sizeof(double) * 2 * m), *b = (double *)malloc(sizeof(double) * 2 * m);
    for (size_t j = 0; j < 2 * m; ++j) a[j] = b[j] = rnd(&s);
    for (int ax = 0; ax < 3; ++ax) expect(kgo_fft3d_axis(nx, ny, nz, a, ax, -1) == 0, "fft3d_axis");
    expect(kgo_fft3d(nx, ny, nz, a, 1) == 0, "fft3d");
    double err = 0;
    for (size_t j = 0; j < 2 * m; ++j) err = fmax(err, fabs(a[j] / (double)m - b[j]));
    expect(err < 1e-12, "fft3d round trip");
    expect(kgo_fft1d(0, a, -1) != 0 && kgo_fft1d(4, a, 0) != 0 && kgo_fft1d(4, NULL, 1) != 0,
           "fft1d rejects");
    expect(kgo_fft3d_axis(nx, ny, nz, a, 3, -1) != 0, "fft3d_axis rejects");
    free(a);
    free(b);
}

static void runs(void)
{
    const double L = 8.0 * M_PI;
    for (int n = 8; n <= 12; n += 4) {  /* radix 2, and lines of 12 (a factor 3) */
        const size_t M = (size_t)n * n * n;
        double *u0 = field(n, 0.3, 11), *aux = field(n, 0.3, 12);
        double *u = (double *)malloc(sizeof(double) * M), *up = (double *)malloc(sizeof(double) * M);
        const int steps = 6;
        double E[7], mx[7], q4[7], secs;
        int blow;
        for (int lin = 0; lin < 2; ++lin)
            for (int deal = 0; deal < 2; ++deal)
                for (int mode = 0; mode < 2; ++mode) {
                    int rc = kgo_run(n, n, n, L, L, L, 0.01, lin, deal, 1e3, mode, u0,
                                     mode ? aux : NULL, steps, u, up, E, mx, q4, &blow, &secs);
                    expect(rc == 0 && blow < 0 && isfinite(E[steps]), "kgo_run");
                    rc = kgo_run(n, n, n, L, L, L, 0.01, lin, deal, 0.0, mode, u0,
                                 mode ? aux : NULL, steps, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
                    expect(rc == 0, "kgo_run without outputs");
                }
        double *vp = (double *)malloc(sizeof(double) * 2 * M), *vc = (double *)malloc(sizeof(double) * 2 * M);
        expect(kgo_state(n, n, n, L, L, L, 0.01, 0, 0, 0, u0, NULL, 4, vp, vc) == 0, "kgo_state");
        expect(kgo_state(n, n, n, L, L, L, 0.01, 0, 1, 1, u0, aux, 4, vp, vc) == 0, "kgo_state two-level");
        const int modes[] = {0, 0, 0, 1, 2, 3, n - 1, n / 2, 1};
        double v0[6], v1[6];
        expect(kgo_first_step_modes(n, n, n, L, L, L, 0.01, 0, u0, 3, modes, v0, v1) == 0,
               "kgo_first_step_modes");
        /* complex field: the same real data as real and imaginary parts */
        double *c0 = (double *)malloc(sizeof(double) * 2 * M), *cu = (double *)malloc(sizeof(double) * 2 * M);
        for (size_t j = 0; j < M; ++j) {
            c0[2 * j] = u0[j];
            c0[2 * j + 1] = 0.5 * aux[j];
        }
        for (int deal = 0; deal < 2; ++deal)
            expect(kgo_run_c(n, n, n, L, L, L, 0.01, 0, deal, 1e3, 0, c0, NULL, steps, cu, NULL, E,
                             mx, q4, &blow) == 0 && blow < 0, "kgo_run_c");
        /* a blow-up: uniform a = 1.5 crosses 1e3 at step 145 with dt = 0.01 */
        for (size_t j = 0; j < M; ++j) u0[j] = 1.5;
        double Eb[201], mb[201], qb[201];
        expect(kgo_run(n, n, n, L, L, L, 0.01, 0, 0, 1e3, 0, u0, NULL, 200, u, up, Eb, mb, qb, &blow,
                       NULL) == 0 && blow == 145, "blow-up step");
        /* rejected arguments */
        expect(kgo_run(n + 1, n, n, L, L, L, 0.01, 0, 0, 1e3, 0, u0, NULL, 2, NULL, NULL, NULL, NULL,
                       NULL, NULL, NULL) != 0, "odd n rejected");
        expect(kgo_run(n, n, n, L, L, L, -0.01, 0, 0, 1e3, 0, u0, NULL, 2, NULL, NULL, NULL, NULL,
                       NULL, NULL, NULL) != 0, "dt <= 0 rejected");
        expect(kgo_run(n, n, n, L, L, L, 0.01, 0, 0, 1e3, 1, u0, NULL, 2, NULL, NULL, NULL, NULL,
                       NULL, NULL, NULL) != 0, "two-level start without u^-1 rejected");
        expect(kgo_run(n, n, n, L, L, L, 0.01, 0, 0, 1e3, 0, NULL, NULL, 2, NULL, NULL, NULL, NULL,
                       NULL, NULL, NULL) != 0, "missing u0 rejected");
        free(u0);
        free(aux);
        free(u);
        free(up);
        free(vp);
        free(vc);
        free(c0);
        free(cu);
    }
}

int main(void)
{
    expect(kgo_num_threads() >= 1, "threads");
    transforms();
    runs();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
