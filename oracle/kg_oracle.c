/*
 * kg_oracle.c -- TEST INFRASTRUCTURE, not part of the solver library.
 *
 * A plain, slow, double-precision CPU reference for the Fourier pseudo-spectral
 * solution of the real cubic Klein-Gordon equation
 *
 *     u_tt - Lap(u) + u = u^3                       (Sec. 1, eq. (1), real u)
 *
 * on a periodic box, stepped with the second-order semi-implicit scheme of
 * Sec. 1.1.2, eq. (2), where time stepping happens in Fourier space and the
 * cubic term is formed in physical space (Sec. 1.1.2, closing paragraph).
 * kgo_run_c steps a complex field, for which the cubic term is |u|^2 u
 * (Sec. 1); it reduces to kgo_run for real data.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code, header, table or helper
 * with the GPU implementation; it has its own FFT (a recursive mixed-radix
 * Cooley-Tukey transform on whole lines, with a twiddle table built from
 * cos/sin) and runs every step on the full complex spectrum.
 *
 * Conventions (the paper does not fix them; the readings are listed with the
 * design notes of the project):
 *   - fields are stored [z][y][x], x fastest;
 *   - forward transform   X[k] = sum_j x[j] exp(-2 pi i j k / n), unnormalised;
 *   - inverse transform   x[j] = sum_k X[k] exp(+2 pi i j k / n), unnormalised;
 *     the 1/M of the inverse (M = nx*ny*nz) is applied explicitly;
 *   - mode index i along an axis of n points has integer wavenumber m = i for
 *     i <= n/2 and m = i - n above, and k = 2 pi m / L; only |k|^2 is used.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC kg_oracle.c -o libkg_oracle.so -lm
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define KGO_OK 0
#define KGO_EINVAL 1
#define KGO_ENOMEM 3

#define KGO_INIT_VELOCITY 0
#define KGO_INIT_TWO_LEVEL 1

int kgo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* One-dimensional DFT                                                        */
/* ------------------------------------------------------------------------- */

/* tw[j] = exp(sign * 2 pi i j / n), j < n, each entry from cos/sin directly. */
static cplx *twiddle_table(int n, int sign)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!tw)
        return NULL;
    for (int j = 0; j < n; j++) {
        double ang = 2.0 * M_PI * (double)j / (double)n;
        tw[j] = cos(ang) + (double)sign * sin(ang) * I;
    }
    return tw;
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; p++)
        if (n % p == 0)
            return p;
    return n;
}

/*
 * Decimation in time.  Computes, for k < n,
 *     out[k] = sum_{j<n} in[j*is] * w^(j*k*ts),   w = tw[1], ts = N/n,
 * where tw is the table of the N-th roots of unity for the full line length N.
 * The input is split into p interleaved subsequences (p the smallest prime
 * factor of n); their length-n/p transforms are combined with
 *     X[k1 + s*m] = sum_r w_p^(r*s) * ( w_n^(r*k1) * Y_r[k1] ).
 */
static void dft_rec(int n, const cplx *in, ptrdiff_t is, cplx *out,
                    const cplx *tw, int N, int ts)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    for (int r = 0; r < p; r++)
        dft_rec(m, in + r * is, is * p, out + (ptrdiff_t)r * m, tw, N, ts * p);

    cplx ybuf[16];
    cplx *y = (p <= 16) ? ybuf : (cplx *)malloc(sizeof(cplx) * (size_t)p);
    for (int k1 = 0; k1 < m; k1++) {
        for (int r = 0; r < p; r++)
            y[r] = out[(ptrdiff_t)r * m + k1] * tw[(r * k1 * ts) % N];
        for (int s = 0; s < p; s++) {
            cplx acc = 0.0;
            for (int r = 0; r < p; r++)
                acc += y[r] * tw[((r * s) % p) * (N / p)];
            out[k1 + (ptrdiff_t)s * m] = acc;
        }
    }
    if (y != ybuf)
        free(y);
}

/* In-place unnormalised DFT of one contiguous line; sign -1 forward, +1 inverse. */
int kgo_fft1d(int n, double *data, int sign)
{
    if (n < 1 || (sign != 1 && sign != -1) || !data)
        return KGO_EINVAL;
    cplx *x = (cplx *)data;
    cplx *tw = twiddle_table(n, sign);
    cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!tw || !out) {
        free(tw);
        free(out);
        return KGO_ENOMEM;
    }
    dft_rec(n, x, 1, out, tw, n, 1);
    memcpy(x, out, sizeof(cplx) * (size_t)n);
    free(tw);
    free(out);
    return KGO_OK;
}

/* ------------------------------------------------------------------------- */
/* Three-dimensional DFT, one axis at a time                                  */
/* ------------------------------------------------------------------------- */

/* Transform every line along `axis` (0 = x, 1 = y, 2 = z) of a [z][y][x] array. */
static int fft3d_axis(int nx, int ny, int nz, cplx *a, int axis, int sign)
{
    int n = axis == 0 ? nx : axis == 1 ? ny : nz;
    ptrdiff_t stride = axis == 0 ? 1 : axis == 1 ? (ptrdiff_t)nx : (ptrdiff_t)nx * ny;
    long nlines = (long)nx * ny * nz / n;
    cplx *tw = twiddle_table(n, sign);
    if (!tw)
        return KGO_ENOMEM;
    int err = 0;
#pragma omp parallel
    {
        cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        if (!line || !out) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long l = 0; l < nlines; l++) {
                ptrdiff_t base;
                if (axis == 0)
                    base = (ptrdiff_t)l * nx;
                else if (axis == 1)
                    base = (ptrdiff_t)(l / nx) * nx * ny + (l % nx);
                else
                    base = (ptrdiff_t)l;
                for (int j = 0; j < n; j++)
                    line[j] = a[base + j * stride];
                dft_rec(n, line, 1, out, tw, n, 1);
                for (int j = 0; j < n; j++)
                    a[base + j * stride] = out[j];
            }
        }
        free(line);
        free(out);
    }
    free(tw);
    return err ? KGO_ENOMEM : KGO_OK;
}

int kgo_fft3d_axis(int nx, int ny, int nz, double *data, int axis, int sign)
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || (sign != 1 && sign != -1) || !data)
        return KGO_EINVAL;
    return fft3d_axis(nx, ny, nz, (cplx *)data, axis, sign);
}

/* Full unnormalised 3D DFT in place (x, then y, then z). */
int kgo_fft3d(int nx, int ny, int nz, double *data, int sign)
{
    int e;
    for (int ax = 0; ax < 3; ax++)
        if ((e = kgo_fft3d_axis(nx, ny, nz, data, ax, sign)) != KGO_OK)
            return e;
    return KGO_OK;
}

/* ------------------------------------------------------------------------- */
/* Klein-Gordon stepping, eq. (2) in Fourier space                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, nz;
    double Lx, Ly, Lz;
    double dt;
    double chi; /* 1 with the cubic term, 0 for the linear equation */
    int dealias; /* nonzero: 2/3-rule truncation of the nonlinear term */
} grid_t;

/* Signed integer wavenumber of mode index i on an axis of n points. */
static int mode_number(int i, int n) { return i <= n / 2 ? i : i - n; }

/*
 * Optional dealiasing, an addition to the paper's plain pseudo-spectral
 * method (which has none): the 2/3 rule applied to the nonlinear term.  A
 * mode is kept when its wavenumber satisfies |m| <= n/3 (integer division)
 * on every axis; the transformed nonlinear term is zeroed on all other modes
 * before the update, so those evolve under the linear part of eq. (2) only.
 */
static int kept_mode(const grid_t *g, int ix, int iy, int iz)
{
    return abs(mode_number(ix, g->nx)) <= g->nx / 3 && abs(mode_number(iy, g->ny)) <= g->ny / 3 &&
           abs(mode_number(iz, g->nz)) <= g->nz / 3;
}

static void truncate_nonlinear(const grid_t *g, cplx *w)
{
    if (!g->dealias)
        return;
    int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int iz = 0; iz < nz; iz++)
        for (int iy = 0; iy < ny; iy++)
            for (int ix = 0; ix < nx; ix++)
                if (!kept_mode(g, ix, iy, iz))
                    w[((size_t)iz * ny + iy) * nx + ix] = 0.0;
}

/* omega_k^2 = 1 + |k|^2: the Fourier symbol of (1 - Lap). */
static double omega2(const grid_t *g, int ix, int iy, int iz)
{
    double kx = 2.0 * M_PI * mode_number(ix, g->nx) / g->Lx;
    double ky = 2.0 * M_PI * mode_number(iy, g->ny) / g->Ly;
    double kz = 2.0 * M_PI * mode_number(iz, g->nz) / g->Lz;
    return 1.0 + kx * kx + ky * ky + kz * kz;
}

/*
 * Eq. (2) transformed: with a = omega^2 dt^2 / 4 each Fourier mode obeys
 *   (1+a) v^{n+1} - 2(1-a) v^n + (1+a) v^{n-1} = dt^2 N^n,
 * so v^{n+1} = alpha v^n - v^{n-1} + beta N^n with
 *   alpha = 2(1-a)/(1+a),  beta = dt^2/(1+a).
 */
static void scheme_coeffs(const grid_t *g, int ix, int iy, int iz, double *alpha, double *beta)
{
    double a = omega2(g, ix, iy, iz) * g->dt * g->dt / 4.0;
    *alpha = 2.0 * (1.0 - a) / (1.0 + a);
    *beta = g->dt * g->dt / (1.0 + a);
}

static size_t npts(const grid_t *g) { return (size_t)g->nx * g->ny * g->nz; }

/* dst = F[src] for a real field src. */
static int forward_real(const grid_t *g, const double *src, cplx *dst)
{
    size_t M = npts(g);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < M; i++)
        dst[i] = src[i];
    return fft3d_axis(g->nx, g->ny, g->nz, dst, 0, -1) ||
           fft3d_axis(g->nx, g->ny, g->nz, dst, 1, -1) ||
           fft3d_axis(g->nx, g->ny, g->nz, dst, 2, -1);
}

/* work = F^{-1}[v] / M, real part kept in u (u may be NULL).  Returns the
 * statistics of the physical field: max|u|, h^3 sum u^4 and a non-finite flag. */
typedef struct {
    double maxabs, q4;
    int nonfinite;
} fieldstats_t;

static int physical(const grid_t *g, const cplx *v, cplx *work, double *u, fieldstats_t *st)
{
    size_t M = npts(g);
    memcpy(work, v, sizeof(cplx) * M);
    int e = fft3d_axis(g->nx, g->ny, g->nz, work, 0, 1) ||
            fft3d_axis(g->nx, g->ny, g->nz, work, 1, 1) ||
            fft3d_axis(g->nx, g->ny, g->nz, work, 2, 1);
    if (e)
        return KGO_ENOMEM;
    double h3 = (g->Lx / g->nx) * (g->Ly / g->ny) * (g->Lz / g->nz);
    double mx = 0.0, s4 = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : mx) reduction(+ : s4) reduction(| : bad)
    for (size_t i = 0; i < M; i++) {
        double x = creal(work[i]) / (double)M;
        work[i] = x; /* the field is real: the imaginary part is dropped */
        if (u)
            u[i] = x;
        if (!isfinite(x))
            bad |= 1;
        double ax = fabs(x);
        if (ax > mx)
            mx = ax;
        s4 += x * x * x * x;
    }
    st->maxabs = mx;
    st->q4 = h3 * s4;
    st->nonfinite = bad;
    return KGO_OK;
}

/*
 * Linear part of the discrete energy between levels n and n+1, the energy of
 * Sec. 1.1 with u_t -> (u^{n+1}-u^n)/dt and u -> (u^{n+1}+u^n)/2, evaluated by
 * Parseval (sum_j |f_j|^2 = (1/M) sum_k |F_k|^2, and -Lap -> |k|^2):
 *   (h^3 / (2M)) sum_k [ |v1-v0|^2/dt^2 + omega_k^2 |v1+v0|^2 / 4 ].
 */
static double linear_energy(const grid_t *g, const cplx *v0, const cplx *v1)
{
    double h3 = (g->Lx / g->nx) * (g->Ly / g->ny) * (g->Lz / g->nz);
    double M = (double)npts(g);
    double s = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : s)
    for (int iz = 0; iz < g->nz; iz++)
        for (int iy = 0; iy < g->ny; iy++)
            for (int ix = 0; ix < g->nx; ix++) {
                size_t i = ((size_t)iz * g->ny + iy) * g->nx + ix;
                double w2 = omega2(g, ix, iy, iz);
                cplx d = v1[i] - v0[i];
                cplx p = v1[i] + v0[i];
                double dd = creal(d) * creal(d) + cimag(d) * cimag(d);
                double pp = creal(p) * creal(p) + cimag(p) * cimag(p);
                s += dd / (g->dt * g->dt) + w2 * pp / 4.0;
            }
    return h3 / (2.0 * M) * s;
}

/*
 * Initial levels (v^{-1}, v^0) from the initial data.  Eq. (2) needs two
 * time levels; the paper does not say how the second one is obtained.
 * Mode KGO_INIT_VELOCITY takes aux = u_t(0) (NULL means zero) and starts the
 * scheme symmetrically in time,
 *   v^{-1} = (alpha/2) v^0 - dt F[u_t0] + (beta/2) chi F[(u^0)^3],
 * the level for which the v^1 produced by eq. (2) satisfies
 * (v^1 - v^{-1}) / (2 dt) = F[u_t0] and (v^1 + v^{-1}) / 2 = v^0 + O(dt^2).
 * Mode KGO_INIT_TWO_LEVEL takes aux = u^{-1} itself.
 */
static int init_levels(const grid_t *g, int mode, const double *u0, const double *aux,
                       cplx *vp, cplx *vc, cplx *w, double *cube)
{
    size_t M = npts(g);
    if (forward_real(g, u0, vc))
        return KGO_ENOMEM;
    if (mode == KGO_INIT_TWO_LEVEL)
        return forward_real(g, aux, vp) ? KGO_ENOMEM : KGO_OK;

#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < M; i++)
        cube[i] = g->chi * u0[i] * u0[i] * u0[i];
    if (forward_real(g, cube, w))
        return KGO_ENOMEM;
    truncate_nonlinear(g, w);
    if (aux) {
        if (forward_real(g, aux, vp))
            return KGO_ENOMEM;
    } else {
        memset(vp, 0, sizeof(cplx) * M);
    }
    int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int iz = 0; iz < nz; iz++)
        for (int iy = 0; iy < ny; iy++)
            for (int ix = 0; ix < nx; ix++) {
                size_t i = ((size_t)iz * ny + iy) * nx + ix;
                double al, be;
                scheme_coeffs(g, ix, iy, iz, &al, &be);
                vp[i] = 0.5 * al * vc[i] - g->dt * vp[i] + 0.5 * be * w[i];
            }
    return KGO_OK;
}

/*
 * One step of eq. (2) given u^n (real, in `cube`, overwritten):
 *   N^n = chi F[(u^n)^3];  v^{n+1} = alpha v^n - v^{n-1} + beta N^n,
 * with v^{n+1} written over v^{n-1} (in vp).
 */
static int advance(const grid_t *g, cplx *vp, const cplx *vc, cplx *w, double *cube)
{
    size_t M = npts(g);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < M; i++)
        cube[i] = g->chi * cube[i] * cube[i] * cube[i];
    if (forward_real(g, cube, w))
        return KGO_ENOMEM;
    truncate_nonlinear(g, w);
    int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int iz = 0; iz < nz; iz++)
        for (int iy = 0; iy < ny; iy++)
            for (int ix = 0; ix < nx; ix++) {
                size_t i = ((size_t)iz * ny + iy) * nx + ix;
                double al, be;
                scheme_coeffs(g, ix, iy, iz, &al, &be);
                vp[i] = al * vc[i] - vp[i] + be * w[i];
            }
    return KGO_OK;
}

static int check_args(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
                      int mode, const double *u0, const double *aux, int nsteps)
{
    if (nx < 2 || ny < 2 || nz < 2 || ((nx | ny | nz) & 1) || !(dt > 0) || !(Lx > 0) ||
        !(Ly > 0) || !(Lz > 0) || !u0 || nsteps < 0 ||
        (mode != KGO_INIT_VELOCITY && mode != KGO_INIT_TWO_LEVEL) ||
        (mode == KGO_INIT_TWO_LEVEL && !aux))
        return KGO_EINVAL;
    return KGO_OK;
}

/*
 * Run `nsteps` steps of eq. (2) from the initial data and report, for the
 * levels n = 0..nsteps (or up to blow-up):
 *   maxu[n]   = max_j |u^n_j| (NaN if u^n has a non-finite value),
 *   q4[n]     = h^3 sum_j (u^n_j)^4,
 *   energy[0] = E^{-1/2}, energy[n+1] = E^{n+1/2} for n < nsteps, where
 *     E^{n+1/2} = linear_energy(v^n, v^{n+1}) - chi (q4[n] + q4[n+1]) / 8
 *   (the quartic term of the Sec. 1.1 energy averaged over the two levels);
 *   u_out     = u^{nsteps}, or the level at which blow-up was detected;
 *   uprev_out = the level before u_out;
 *   *blowup_step = first n with max|u^n| > threshold or a non-finite value,
 *                  -1 if none (threshold <= 0 disables the test);
 *   *loop_seconds = wall time of the steps themselves (levels 0..nsteps-1:
 *                  inverse transform, cubic term, forward transform, update),
 *                  without the set-up and the last level's transform.
 * dealias nonzero truncates the nonlinear term by the 2/3 rule (kept_mode).
 * Any output pointer may be NULL.  Entries after a blow-up stay NaN.
 */
static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int kgo_run(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
            int linear_only, int dealias, double threshold, int mode,
            const double *u0, const double *aux, int nsteps,
            double *u_out, double *uprev_out,
            double *energy, double *maxu, double *q4, int *blowup_step,
            double *loop_seconds)
{
    int rc = check_args(nx, ny, nz, Lx, Ly, Lz, dt, mode, u0, aux, nsteps);
    if (rc != KGO_OK)
        return rc;

    grid_t g = {nx, ny, nz, Lx, Ly, Lz, dt, linear_only ? 0.0 : 1.0, dealias != 0};
    size_t M = npts(&g);
    cplx *vp = (cplx *)malloc(sizeof(cplx) * M);   /* v^{n-1} */
    cplx *vc = (cplx *)malloc(sizeof(cplx) * M);   /* v^n     */
    cplx *w = (cplx *)malloc(sizeof(cplx) * M);    /* work    */
    double *cube = (double *)malloc(sizeof(double) * M);
    int blown = -1;
    fieldstats_t st;
    if (!vp || !vc || !w || !cube) {
        rc = KGO_ENOMEM;
        goto done;
    }
    for (int n = 0; n <= nsteps; n++) {
        if (maxu) maxu[n] = NAN;
        if (q4) q4[n] = NAN;
        if (energy) energy[n] = NAN;
    }
    if ((rc = init_levels(&g, mode, u0, aux, vp, vc, w, cube)) != KGO_OK)
        goto done;

    /* E^{-1/2} needs the quartic sums of u^{-1} and u^0. */
    if ((rc = physical(&g, vp, w, NULL, &st)) != KGO_OK)
        goto done;
    double q4_prev = st.q4;
    double elin_prev = linear_energy(&g, vp, vc);

    double t0 = wall_seconds(), t1 = t0;
    for (int n = 0; n <= nsteps; n++) {
        if (n == nsteps)
            t1 = wall_seconds();  /* the last level's transform is output, not a step */
        /* u^n = Re F^{-1}[v^n] / M; its statistics decide blow-up. */
        if ((rc = physical(&g, vc, w, cube, &st)) != KGO_OK)
            goto done;
        if (maxu) maxu[n] = st.nonfinite ? NAN : st.maxabs;
        if (q4) q4[n] = st.q4;
        if (energy) energy[n] = elin_prev - g.chi * (q4_prev + st.q4) / 8.0;
        int is_blown = st.nonfinite || (threshold > 0 && st.maxabs > threshold);
        if (is_blown || n == nsteps) {
            if (is_blown) blown = n;
            if (u_out) memcpy(u_out, cube, sizeof(double) * M);
            break;
        }
        if ((rc = advance(&g, vp, vc, w, cube)) != KGO_OK)
            goto done;
        elin_prev = linear_energy(&g, vc, vp);
        q4_prev = st.q4;
        cplx *t = vp; vp = vc; vc = t; /* vc = v^{n+1}, vp = v^n */
    }
    if (uprev_out)
        rc = physical(&g, vp, w, uprev_out, &st);
    if (loop_seconds)
        *loop_seconds = t1 > t0 ? t1 - t0 : 0.0;

done:
    if (blowup_step) *blowup_step = blown;
    free(vp); free(vc); free(w); free(cube);
    return rc;
}

/*
 * Spectral levels after `nsteps` steps, without the blow-up test: the full
 * complex spectra v^{nsteps-1} (v_prev) and v^{nsteps} (v_cur), interleaved
 * re/im in [z][y][x] order.
 */
int kgo_state(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
              int linear_only, int dealias, int mode, const double *u0, const double *aux,
              int nsteps, double *v_prev, double *v_cur)
{
    int rc = check_args(nx, ny, nz, Lx, Ly, Lz, dt, mode, u0, aux, nsteps);
    if (rc != KGO_OK || !v_prev || !v_cur)
        return rc != KGO_OK ? rc : KGO_EINVAL;
    grid_t g = {nx, ny, nz, Lx, Ly, Lz, dt, linear_only ? 0.0 : 1.0, dealias != 0};
    size_t M = npts(&g);
    cplx *vp = (cplx *)malloc(sizeof(cplx) * M);
    cplx *vc = (cplx *)malloc(sizeof(cplx) * M);
    cplx *w = (cplx *)malloc(sizeof(cplx) * M);
    double *cube = (double *)malloc(sizeof(double) * M);
    fieldstats_t st;
    if (!vp || !vc || !w || !cube) {
        rc = KGO_ENOMEM;
        goto done;
    }
    if ((rc = init_levels(&g, mode, u0, aux, vp, vc, w, cube)) != KGO_OK)
        goto done;
    for (int n = 0; n < nsteps; n++) {
        if ((rc = physical(&g, vc, w, cube, &st)) != KGO_OK)
            goto done;
        if ((rc = advance(&g, vp, vc, w, cube)) != KGO_OK)
            goto done;
        cplx *t = vp; vp = vc; vc = t;
    }
    memcpy(v_prev, vp, sizeof(cplx) * M);
    memcpy(v_cur, vc, sizeof(cplx) * M);
done:
    free(vp); free(vc); free(w); free(cube);
    return rc;
}

/*
 * The first step of eq. (2) at selected modes, from u(0) = u0 and u_t(0) = 0,
 * by direct summation of the DFT definition at each mode k (index triple
 * (ix, iy, iz), 0 <= i < n per axis):
 *   v^0_k = sum_j u0_j exp(-2 pi i (ix jx/nx + iy jy/ny + iz jz/nz)),
 *   N^0_k = chi * (the same sum of u0_j^3),
 *   v^{-1}_k = (alpha/2) v^0_k + (beta/2) N^0_k     (symmetric start, u_t = 0),
 *   v^1_k = alpha v^0_k - v^{-1}_k + beta N^0_k.
 * Lets a solver's output at any grid size be checked mode by mode.
 * v0_out and v1_out receive 2*nmodes doubles (re, im).
 */
int kgo_first_step_modes(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
                         int linear_only, const double *u0, int nmodes, const int *modes,
                         double *v0_out, double *v1_out)
{
    if (check_args(nx, ny, nz, Lx, Ly, Lz, dt, KGO_INIT_VELOCITY, u0, NULL, 0) != KGO_OK ||
        nmodes < 0 || (nmodes && (!modes || !v0_out || !v1_out)))
        return KGO_EINVAL;
    grid_t g = {nx, ny, nz, Lx, Ly, Lz, dt, linear_only ? 0.0 : 1.0};
    cplx *ex = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    cplx *ey = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
    cplx *ez = (cplx *)malloc(sizeof(cplx) * (size_t)nz);
    if (!ex || !ey || !ez) {
        free(ex); free(ey); free(ez);
        return KGO_ENOMEM;
    }
    for (int q = 0; q < nmodes; q++) {
        int ix = modes[3 * q], iy = modes[3 * q + 1], iz = modes[3 * q + 2];
        if (ix < 0 || ix >= nx || iy < 0 || iy >= ny || iz < 0 || iz >= nz) {
            free(ex); free(ey); free(ez);
            return KGO_EINVAL;
        }
        for (int j = 0; j < nx; j++) {
            double a = -2.0 * M_PI * (double)(((long)ix * j) % nx) / nx;
            ex[j] = cos(a) + sin(a) * I;
        }
        for (int j = 0; j < ny; j++) {
            double a = -2.0 * M_PI * (double)(((long)iy * j) % ny) / ny;
            ey[j] = cos(a) + sin(a) * I;
        }
        for (int j = 0; j < nz; j++) {
            double a = -2.0 * M_PI * (double)(((long)iz * j) % nz) / nz;
            ez[j] = cos(a) + sin(a) * I;
        }
        double r1 = 0, i1 = 0, r3 = 0, i3 = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : r1, i1, r3, i3)
        for (int jz = 0; jz < nz; jz++)
            for (int jy = 0; jy < ny; jy++) {
                const double *row = u0 + ((size_t)jz * ny + jy) * nx;
                cplx s1 = 0, s3 = 0;
                for (int jx = 0; jx < nx; jx++) {
                    double u = row[jx];
                    s1 += u * ex[jx];
                    s3 += u * u * u * ex[jx];
                }
                cplx f = ey[jy] * ez[jz];
                s1 *= f;
                s3 *= f;
                r1 += creal(s1); i1 += cimag(s1);
                r3 += creal(s3); i3 += cimag(s3);
            }
        cplx v0 = r1 + i1 * I, nl = g.chi * (r3 + i3 * I);
        double al, be;
        scheme_coeffs(&g, ix, iy, iz, &al, &be);
        cplx vm1 = 0.5 * al * v0 + 0.5 * be * nl;
        cplx v1 = al * v0 - vm1 + be * nl;
        v0_out[2 * q] = creal(v0); v0_out[2 * q + 1] = cimag(v0);
        v1_out[2 * q] = creal(v1); v1_out[2 * q + 1] = cimag(v1);
    }
    free(ex); free(ey); free(ez);
    return KGO_OK;
}

/* ------------------------------------------------------------------------- */
/* Complex fields                                                             */
/* ------------------------------------------------------------------------- */

/*
 * The benchmark code of the paper also allows a complex field (Sec. 1.1.2);
 * the cubic term of eq. (1) is then |u|^2 u (Sec. 1), which reduces to u^3
 * for real u.  Fields are complex [z][y][x] arrays, interleaved re/im.
 */

/* dst = F[src] for a complex field src. */
static int forward_cplx(const grid_t *g, const cplx *src, cplx *dst)
{
    memcpy(dst, src, sizeof(cplx) * npts(g));
    return fft3d_axis(g->nx, g->ny, g->nz, dst, 0, -1) ||
           fft3d_axis(g->nx, g->ny, g->nz, dst, 1, -1) ||
           fft3d_axis(g->nx, g->ny, g->nz, dst, 2, -1);
}

/* u = F^{-1}[v] / M, complex; statistics max|u|, h^3 sum |u|^4, non-finite. */
static int physical_cplx(const grid_t *g, const cplx *v, cplx *u, fieldstats_t *st)
{
    size_t M = npts(g);
    memcpy(u, v, sizeof(cplx) * M);
    if (fft3d_axis(g->nx, g->ny, g->nz, u, 0, 1) || fft3d_axis(g->nx, g->ny, g->nz, u, 1, 1) ||
        fft3d_axis(g->nx, g->ny, g->nz, u, 2, 1))
        return KGO_ENOMEM;
    double h3 = (g->Lx / g->nx) * (g->Ly / g->ny) * (g->Lz / g->nz);
    double mx = 0.0, s4 = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : mx) reduction(+ : s4) reduction(| : bad)
    for (size_t i = 0; i < M; i++) {
        cplx x = u[i] / (double)M;
        u[i] = x;
        double m2 = creal(x) * creal(x) + cimag(x) * cimag(x);
        if (!isfinite(creal(x)) || !isfinite(cimag(x)))
            bad |= 1;
        if (sqrt(m2) > mx)
            mx = sqrt(m2);
        s4 += m2 * m2;
    }
    st->maxabs = mx;
    st->q4 = h3 * s4;
    st->nonfinite = bad;
    return KGO_OK;
}

/* w = chi F[|u|^2 u]. */
static int nonlinear_cplx(const grid_t *g, const cplx *u, cplx *w, cplx *tmp)
{
    size_t M = npts(g);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < M; i++) {
        double m2 = creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
        tmp[i] = g->chi * m2 * u[i];
    }
    if (forward_cplx(g, tmp, w))
        return KGO_ENOMEM;
    truncate_nonlinear(g, w);
    return KGO_OK;
}

/*
 * kgo_run for a complex field: u0 and aux (u_t(0) or u^{-1}, may be NULL in
 * velocity mode) are complex; the nonlinear term is chi |u|^2 u; u_out and
 * uprev_out receive complex fields; maxu[n] = max_j |u^n_j|,
 * q4[n] = h^3 sum_j |u^n_j|^4 and the energy is that of kgo_run (the same
 * expression with |.|, equal to it for real data).  Start rules as in
 * init_levels, with |u0|^2 u0 for u0^3.
 */
int kgo_run_c(int nx, int ny, int nz, double Lx, double Ly, double Lz, double dt,
              int linear_only, int dealias, double threshold, int mode,
              const double *u0, const double *aux, int nsteps,
              double *u_out, double *uprev_out,
              double *energy, double *maxu, double *q4, int *blowup_step)
{
    int rc = check_args(nx, ny, nz, Lx, Ly, Lz, dt, mode, u0, aux, nsteps);
    if (rc != KGO_OK)
        return rc;
    grid_t g = {nx, ny, nz, Lx, Ly, Lz, dt, linear_only ? 0.0 : 1.0, dealias != 0};
    size_t M = npts(&g);
    cplx *vp = (cplx *)malloc(sizeof(cplx) * M);
    cplx *vc = (cplx *)malloc(sizeof(cplx) * M);
    cplx *w = (cplx *)malloc(sizeof(cplx) * M);
    cplx *u = (cplx *)malloc(sizeof(cplx) * M);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * M);
    int blown = -1;
    fieldstats_t st;
    if (!vp || !vc || !w || !u || !tmp) {
        rc = KGO_ENOMEM;
        goto done;
    }
    for (int n = 0; n <= nsteps; n++) {
        if (maxu) maxu[n] = NAN;
        if (q4) q4[n] = NAN;
        if (energy) energy[n] = NAN;
    }
    /* initial levels */
    if (forward_cplx(&g, (const cplx *)u0, vc)) {
        rc = KGO_ENOMEM;
        goto done;
    }
    if (mode == KGO_INIT_TWO_LEVEL) {
        if (forward_cplx(&g, (const cplx *)aux, vp)) {
            rc = KGO_ENOMEM;
            goto done;
        }
    } else {
        if (nonlinear_cplx(&g, (const cplx *)u0, w, tmp)) {
            rc = KGO_ENOMEM;
            goto done;
        }
        if (aux) {
            if (forward_cplx(&g, (const cplx *)aux, vp)) {
                rc = KGO_ENOMEM;
                goto done;
            }
        } else {
            memset(vp, 0, sizeof(cplx) * M);
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int iz = 0; iz < nz; iz++)
            for (int iy = 0; iy < ny; iy++)
                for (int ix = 0; ix < nx; ix++) {
                    size_t i = ((size_t)iz * ny + iy) * nx + ix;
                    double al, be;
                    scheme_coeffs(&g, ix, iy, iz, &al, &be);
                    vp[i] = 0.5 * al * vc[i] - g.dt * vp[i] + 0.5 * be * w[i];
                }
    }
    if ((rc = physical_cplx(&g, vp, u, &st)) != KGO_OK)
        goto done;
    double q4_prev = st.q4;
    double elin_prev = linear_energy(&g, vp, vc);
    for (int n = 0; n <= nsteps; n++) {
        if ((rc = physical_cplx(&g, vc, u, &st)) != KGO_OK)
            goto done;
        if (maxu) maxu[n] = st.nonfinite ? NAN : st.maxabs;
        if (q4) q4[n] = st.q4;
        if (energy) energy[n] = elin_prev - g.chi * (q4_prev + st.q4) / 8.0;
        int is_blown = st.nonfinite || (threshold > 0 && st.maxabs > threshold);
        if (is_blown || n == nsteps) {
            if (is_blown) blown = n;
            if (u_out) memcpy(u_out, u, sizeof(cplx) * M);
            break;
        }
        /* v^{n+1} = alpha v^n - v^{n-1} + beta chi F[|u^n|^2 u^n], over v^{n-1} */
        if (nonlinear_cplx(&g, u, w, tmp)) {
            rc = KGO_ENOMEM;
            goto done;
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int iz = 0; iz < nz; iz++)
            for (int iy = 0; iy < ny; iy++)
                for (int ix = 0; ix < nx; ix++) {
                    size_t i = ((size_t)iz * ny + iy) * nx + ix;
                    double al, be;
                    scheme_coeffs(&g, ix, iy, iz, &al, &be);
                    vp[i] = al * vc[i] - vp[i] + be * w[i];
                }
        elin_prev = linear_energy(&g, vc, vp);
        q4_prev = st.q4;
        cplx *t = vp; vp = vc; vc = t;
    }
    if (uprev_out) {
        if ((rc = physical_cplx(&g, vp, tmp, &st)) != KGO_OK)
            goto done;
        memcpy(uprev_out, tmp, sizeof(cplx) * M);
    }
done:
    if (blowup_step) *blowup_step = blown;
    free(vp); free(vc); free(w); free(u); free(tmp);
    return rc;
}
