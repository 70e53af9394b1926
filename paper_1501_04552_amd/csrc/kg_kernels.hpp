// kg_kernels.hpp -- the per-step kernels of the Klein-Gordon stepper (gfx950).
//
// One time step of eq. (2) (Sec. 1.1.2) is four passes over the half
// spectrum plus a one-workgroup finalize:
//   x pass: per (z, y) line, c2r along x of the working field gives u^n(x);
//           record max|u| and sum u^4; form chi*u^3; r2c along x.
//   y pass: per (z, kx) column, forward c2c along y.
//   z pass: per (ky, kx) column, forward c2c along z gives N^n = F[u^3];
//           v^{n+1} = alpha v^n - v^{n-1} + beta N^n (eq. (2) per mode);
//           energy partials of (v^n, v^{n+1}); store v^{n+1}; inverse c2c
//           along z of v^{n+1}/M.
//   y pass: inverse c2c along y; the result feeds the next step's x pass.
// The two 3D FFTs of a step (Sec. 1.1.2, closing paragraph) are thus split
// over the passes, the inverse one finishing in the next step's x pass.
//
// Layouts (element = cx<T>):
//   Q  working field, [z][y][kx] with kx row pitch P = ntx * W >= n/2+1;
//   S  a time level, tile-native [ky][tile][kz][W] (tile = kx / W), private
//      to the z pass so its loads are contiguous per wavefront.
#pragma once

#include "kg_fft.hpp"

namespace kg {

// Device-side control block and per-level record.
struct Ctl {
    int flag;       // 0 running; 1 blown up; 2 stopped by the energy alarm
    int step;       // levels completed (the stopping level once flag is set)
    int blow_step;  // level at which the run stopped, -1 if none
    int pad;
    double elin_m;  // linear energy of the initial pair (v^{-1}, v^0)
    double q4_m;    // h^3 sum (u^{-1})^4
    double maxu_m;  // max |u^{-1}|
    double e_ref;   // E^{-1/2}, the energy of the initial pair (set by the first step)
    double e_tol;   // energy alarm: relative drift that stops the run (0: off)
    double pad2;
};
struct Rec {
    double elin;  // linear energy of (v^m, v^{m+1})
    double q4;    // h^3 sum (u^m)^4
    double maxu;  // max |u^m| (NaN when non-finite)
    double pad;
};

constexpr int RING = 65536;  // records kept on the device

// max that keeps a NaN once one is seen
__device__ __forceinline__ double nanmax(double a, double b)
{
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// Reduce (max, sum) over a workgroup of NT threads (a power of two) in a
// fixed order and write the pair to out[0], out[1] from thread 0.  Every
// thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ void block_max_sum(double mx, double sm, double *out)
{
    constexpr int WS = NT < 64 ? NT : 64;  // lanes combined by shuffles
    constexpr int NW = NT / WS;            // waves
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, off, WS));
        sm += __shfl_xor(sm, off, WS);
    }
    if constexpr (NW == 1) {
        if (threadIdx.x == 0) {
            out[0] = mx;
            out[1] = sm;
        }
    } else {
        __shared__ double red[2][NW];
        if ((threadIdx.x & (WS - 1)) == 0) {
            red[0][threadIdx.x / WS] = mx;
            red[1][threadIdx.x / WS] = sm;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red[0][0], s = red[1][0];
            for (int i = 1; i < NW; ++i) {
                m = nanmax(m, red[0][i]);
                s += red[1][i];
            }
            out[0] = m;
            out[1] = s;
        }
    }
}

// x where `on`, else 0, selected per component.  Written as one select of
// two complex values, the compiler may turn it into a load through a
// selected address (one of them a local zero), which moves register arrays
// to scratch memory and global loads to flat ones.
template <typename T>
__device__ __forceinline__ cx<T> keep(bool on, cx<T> x)
{
    return mk(on ? x.re : (T)0, on ? x.im : (T)0);
}

// The x and y passes load and store the working field with ordinary
// (cached) accesses: a step runs its y-inverse / x / y-forward chain slab by
// slab of z planes so that each slab's intermediate fields stay in the GPU's
// memory-side cache between the three passes.  (Streaming hints there would
// send every intermediate to HBM; the z pass, which sweeps the whole field,
// keeps them.)

// ---------------------------------------------------------------------------
// x pass
// ---------------------------------------------------------------------------

enum XMode { X_STEP = 0, X_REDUCE = 1, X_R2C = 2, X_C2R = 3, X_GAUSS = 4 };

template <typename T>
struct XArgs {
    cx<T> *Q;
    const cx<T> *tw;      // exp(-2 pi i j / n), j < n
    const double *rin;    // X_R2C: real input [z][y][x]
    const double *rin2;   // X_R2C: if set, the input is rin - rin2
    double *rout;         // X_C2R: real output
    double *part;         // X_STEP / X_REDUCE: (max|u|, sum u^4) per workgroup
    const Ctl *ctl;
    int P;                // row pitch of Q
    long PZ;              // plane pitch of Q
    T chi;                // cubic coefficient (X_STEP; X_R2C / X_GAUSS: 1 cubes the input)
    // X_GAUSS: the input is A exp(-(x^2/sx^2 + y^2/sy^2 + z^2/sz^2)) sampled at
    // x_j = -L/2 + j L / N (same for y, z), computed in place of rin
    double gA, gsx, gsy, gsz, gL;
};

// Two real x-lines u1, u2 are transformed together as one complex line
// z = u1 + i u2 of N points: their half spectra X1, X2 (kx = 0..N/2) give
//   Z[k] = X1[k] + i X2[k],  with X[k] = conj(X[N-k]) for k > N/2
// (imaginary parts of X[0] and X[N/2] dropped: the fields are real), and
// the forward transform Z' of (u1^3 + i u2^3) splits back into
//   W1[k] = (Z'[k] + conj Z'[N-k]) / 2,  W2[k] = (Z'[k] - conj Z'[N-k]) / (2i).
template <typename T, int N>
struct XCfg {
    static constexpr int TPL = Radix<N>::TPL;
    static constexpr int NT = 256;
    static constexpr int PPB = NT / TPL;  // line pairs per workgroup
    // LDS slots of the contiguous lines.  FP64: the XOR swizzle on 2^a lines
    // of >= 256 points (bank conflicts 0.03 of LDS cycles against 0.21 with
    // padding at 512^3, less LDS and fewer registers, same time), else one pad
    // slot per 8 positions.  FP32: plain slots; padding (82 VGPRs) and the
    // swizzle (78 VGPRs: its XORed addresses cannot use immediate offsets) both
    // cost occupancy (5-6 instead of 8 waves per SIMD) that the conflicts (0.40
    // of LDS cycles, 0.02 with the swizzle) do not repay: 0.245 ms plain
    // against 0.265 swizzled, 0.39 with the swizzle forced to 8 waves (spills).
    static constexpr bool SWZ_OK = sizeof(T) == 8 && !Radix<N>::THREE && N >= 256;
    static constexpr int SH = SWZ_OK ? SWZ : (sizeof(T) == 8 ? 3 : 0);
    static constexpr int RS = lslots<N, SH>();
    static constexpr long blocks() { return ((long)N * N / 2 + PPB - 1) / PPB; }
    // complex fields: one line per row, PPB rows per workgroup
    static constexpr long blocks_c() { return ((long)N * N + PPB - 1) / PPB; }
};

// One workgroup's share of the x pass: line pairs blk*PPB .. blk*PPB+PPB-1.
// rows: LDS of XCfg<T, N>::PPB * RS elements; part: the workgroup's partial slot.
template <typename T, int N, int MODE>
__device__ __forceinline__ void xbody(const XArgs<T> &a, long blk, cx<T> *rows, double *part)
{
    using C = XCfg<T, N>;
    constexpr int E = Radix<N>::E, TPL = C::TPL, PPB = C::PPB, RS = C::RS;
    // a pair's threads never span two waves, so its stages sync per wave
    constexpr int XSY = (64 % TPL == 0) ? SYNC_WAVE : SYNC_BLOCK;
    static_assert(E % 2 == 0 && E * TPL == N, "the half-spectrum cases are split by position");
    const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
    const long pr = blk * PPB + l;
    const bool act = pr < (long)N * N / 2;
    cx<T> *r = rows + l * RS;
    cx<T> v[E];
    double mx = 0.0, s4 = 0.0;

    if constexpr (MODE == X_GAUSS) {
        const long l1 = 2 * pr;  // first line of the pair: (z, y) = (l1 / N, l1 % N)
        const double h = a.gL / N;
        const double y1 = -0.5 * a.gL + (double)(l1 % N) * h, z1 = -0.5 * a.gL + (double)(l1 / N) * h;
        const double y2 = -0.5 * a.gL + (double)((l1 + 1) % N) * h;
        const double z2 = -0.5 * a.gL + (double)((l1 + 1) / N) * h;
        const double ry1 = y1 * y1 / (a.gsy * a.gsy) + z1 * z1 / (a.gsz * a.gsz);
        const double ry2 = y2 * y2 / (a.gsy * a.gsy) + z2 * z2 / (a.gsz * a.gsz);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int m = t + j * TPL;
            const double x = -0.5 * a.gL + (double)m * h, rx = x * x / (a.gsx * a.gsx);
            double d1 = act ? a.gA * exp(-(rx + ry1)) : 0.0, d2 = act ? a.gA * exp(-(rx + ry2)) : 0.0;
            if (a.chi != (T)0) {
                d1 = d1 * d1 * d1;
                d2 = d2 * d2 * d2;
            }
            v[j] = mk((T)d1, (T)d2);
        }
    } else if constexpr (MODE == X_R2C) {
        const double *s1 = a.rin + (2 * pr) * N, *s2 = s1 + N;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int m = t + j * TPL;
            double d1 = act ? s1[m] : 0.0, d2 = act ? s2[m] : 0.0;
            if (a.rin2 && act) {
                d1 -= a.rin2[(2 * pr) * N + m];
                d2 -= a.rin2[(2 * pr + 1) * N + m];
            }
            T x1 = (T)d1, x2 = (T)d2;
            if (a.chi != (T)0) {
                x1 = x1 * x1 * x1;
                x2 = x2 * x2 * x2;
            }
            v[j] = mk(x1, x2);
        }
    } else {
        // Loads are unconditional so that all of a thread's are in flight
        // together (under a branch each would wait for its data): lanes past
        // the last pair read pair 0 and drop the values.  Each value is read
        // twice (as X[k] and as conj X[N-k]): cached loads.
        const long prc = act ? pr : 0;
        const cx<T> *q1 = a.Q + (2 * prc / N) * a.PZ + (2 * prc % N) * a.P, *q2 = q1 + a.P;
        cx<T> l1[E], l2[E];
        // k = t + j*TPL lies below N/2 for j < E/2 and above it for j > E/2;
        // for j = E/2 it is N/2 + t (N/2 itself only on thread 0, where both
        // forms below agree once the imaginary parts are dropped)
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int k = t + j * TPL;
            const int m = j < E / 2 ? k : N - k;
            l1[j] = q1[m];
            l2[j] = q2[m];
        }
#pragma unroll
        for (int j = 0; j < E; ++j) {
            cx<T> x1 = l1[j], x2 = l2[j];
            if ((j == 0 || j == E / 2) && t == 0) {  // k = 0, k = N/2
                x1.im = 0;
                x2.im = 0;
            }
            // Z = X1 + i X2 (k <= N/2), conj(X1) + i conj(X2) (k > N/2)
            v[j] = j < E / 2 ? mk(x1.re - x2.im, x1.im + x2.re) : mk(x1.re + x2.im, x2.re - x1.im);
        }
        fft_line<T, N, 1, XSY, C::SH>(v, r, 1, t, a.tw, 1);
        // v[j] = u1[m] + i u2[m], m = t + j*TPL
        if constexpr (MODE == X_C2R) {
            if (act) {
                double *d1 = a.rout + (2 * pr) * N, *d2 = d1 + N;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int m = t + j * TPL;
                    d1[m] = (double)v[j].re;
                    d2[m] = (double)v[j].im;
                }
            }
            return;
        }
        // fmax drops NaNs; a NaN value also makes the sum of fourth powers NaN
        // (all terms are >= 0, so no inf - inf), which restores it below.
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const double u1 = (double)v[j].re, u2 = (double)v[j].im;
            if (act) {
                mx = fmax(mx, fmax(fabs(u1), fabs(u2)));
                const double q1 = u1 * u1, q2 = u2 * u2;
                s4 = fma(q1, q1, fma(q2, q2, s4));
            }
        }
        if (s4 != s4) mx = s4;
        if constexpr (MODE == X_REDUCE) {
            block_max_sum<256>(mx, s4, part);
            return;
        }
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const T u1 = v[j].re, u2 = v[j].im;
            v[j] = mk(a.chi * (u1 * u1 * u1), a.chi * (u2 * u2 * u2));
        }
        stage_sync<XSY>();
    }
    fft_line<T, N, -1, XSY, C::SH>(v, r, 1, t, a.tw, 1);
    // positions >= N/2 are the partners N-k of the outputs k = 1..N/2
    stage_sync<XSY>();
#pragma unroll
    for (int j = E / 2; j < E; ++j) {  // k >= N/2
        const int k = t + j * TPL;
        r[lslot<N, C::SH>(k)] = v[j];
    }
    stage_sync<XSY>();
    if (act) {
        cx<T> *q1 = a.Q + (2 * pr / N) * a.PZ + (2 * pr % N) * a.P, *q2 = q1 + a.P;
#pragma unroll
        for (int j = 0; j <= E / 2; ++j) {  // k <= N/2: j < E/2, and k = N/2 on thread 0
            const int k = t + j * TPL;
            if (j < E / 2 || t == 0) {
                const cx<T> zk = v[j];
                const cx<T> zm = (j == 0 && t == 0) ? conjg(zk) : conjg(r[lslot<N, C::SH>(N - k)]);
                q1[k] = scale(zk + zm, (T)0.5);
                q2[k] = scale(rot90<-1>(zk - zm), (T)0.5);
            }
        }
    }
    if constexpr (MODE == X_STEP) block_max_sum<256>(mx, s4, part);
}

// The x pass of a complex field (Sec. 1: the cubic term is |u|^2 u).  Q
// holds the full spectrum, kx = 0..N-1, and each row is one complex line,
// transformed as it stands: no packing of two lines and no Hermitian split.
// The partials are max|u| and sum |u|^4.  Inputs and outputs of X_R2C /
// X_C2R are interleaved (re, im) doubles [z][y][x]; X_GAUSS has no complex
// form.
template <typename T, int N, int MODE>
__device__ __forceinline__ void xbody_c(const XArgs<T> &a, long blk, cx<T> *rows, double *part)
{
    static_assert(MODE != X_GAUSS, "no complex Gaussian input");
    using C = XCfg<T, N>;
    constexpr int E = Radix<N>::E, TPL = C::TPL, PPB = C::PPB, RS = C::RS;
    constexpr int XSY = (64 % TPL == 0) ? SYNC_WAVE : SYNC_BLOCK;
    const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
    const long ln = blk * PPB + l;  // row (z, y) = (ln / N, ln % N)
    const bool act = ln < (long)N * N;
    const long lc = act ? ln : 0;   // lanes past the last row read row 0, store nothing
    cx<T> *r = rows + l * RS;
    cx<T> *q = a.Q + (lc / N) * a.PZ + (lc % N) * a.P;
    cx<T> v[E];
    double mx = 0.0, s4 = 0.0;

    if constexpr (MODE == X_R2C) {
        const double *s = a.rin + 2 * lc * N;
        const double *s2 = a.rin2 ? a.rin2 + 2 * lc * N : nullptr;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int m = t + j * TPL;
            double re = act ? s[2 * m] : 0.0, im = act ? s[2 * m + 1] : 0.0;
            if (s2 && act) {
                re -= s2[2 * m];
                im -= s2[2 * m + 1];
            }
            T xr = (T)re, xi = (T)im;
            if (a.chi != (T)0) {
                const T m2 = xr * xr + xi * xi;
                xr *= m2;
                xi *= m2;
            }
            v[j] = mk(xr, xi);
        }
    } else {
        cx<T> ld[E];
#pragma unroll
        for (int j = 0; j < E; ++j) ld[j] = q[t + j * TPL];
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = ld[j];
        fft_line<T, N, 1, XSY, C::SH>(v, r, 1, t, a.tw, 1);
        // v[j] = u[m], m = t + j*TPL
        if constexpr (MODE == X_C2R) {
            if (act) {
                double *d = a.rout + 2 * ln * N;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int m = t + j * TPL;
                    d[2 * m] = (double)v[j].re;
                    d[2 * m + 1] = (double)v[j].im;
                }
            }
            return;
        }
        // max of |u|^2 (fmax drops NaNs; the sum restores them), then the root
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const double ur = (double)v[j].re, ui = (double)v[j].im;
            if (act) {
                const double m2 = fma(ur, ur, ui * ui);
                mx = fmax(mx, m2);
                s4 = fma(m2, m2, s4);
            }
        }
        if (s4 != s4) mx = s4;
        mx = sqrt(mx);
        if constexpr (MODE == X_REDUCE) {
            block_max_sum<256>(mx, s4, part);
            return;
        }
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const T m2 = v[j].re * v[j].re + v[j].im * v[j].im;
            v[j] = scale(v[j], a.chi * m2);
        }
        stage_sync<XSY>();
    }
    fft_line<T, N, -1, XSY, C::SH>(v, r, 1, t, a.tw, 1);
    if (act) {
#pragma unroll
        for (int j = 0; j < E; ++j) q[t + j * TPL] = v[j];
    }
    if constexpr (MODE == X_STEP) block_max_sum<256>(mx, s4, part);
}

template <typename T, int N, int MODE, bool CF = false>
__global__ __launch_bounds__(256) void k_xpass(XArgs<T> a)
{
    __shared__ cx<T> rows[XCfg<T, N>::PPB * XCfg<T, N>::RS];
    if constexpr (MODE == X_STEP || MODE == X_REDUCE) {
        if (a.ctl->flag) return;
    }
    if constexpr (CF)
        xbody_c<T, N, MODE>(a, blockIdx.x, rows, a.part + 2 * blockIdx.x);
    else
        xbody<T, N, MODE>(a, blockIdx.x, rows, a.part + 2 * blockIdx.x);
}

// ---------------------------------------------------------------------------
// y pass: c2c along y for every (z, kx)
// ---------------------------------------------------------------------------

template <int N, int W>
struct YZCfg {
    static constexpr int TPL = Radix<N>::TPL;
    static constexpr int B0 = 256 / (W * TPL) > 0 ? 256 / (W * TPL) : 1;
    static constexpr int B = B0 < N ? B0 : N;  // outer lines per workgroup
    static constexpr int NT = W * TPL * B;
};

template <typename T>
struct YArgs {
    cx<T> *Q;
    const cx<T> *tw;
    const Ctl *ctl;  // NULL: no blow-up test
    int P, H, ntx;
    long PZ;
};

// One workgroup's tile of the y pass: columns tile*W.. of B consecutive z planes.
template <typename T, int N, int W, int DIR>
__device__ __forceinline__ void ybody(const YArgs<T> &a, long blk, cx<T> *lds)
{
    using C = YZCfg<N, W>;
    constexpr int E = Radix<N>::E, TPL = C::TPL, B = C::B;
    const int c = threadIdx.x % W, t = (threadIdx.x / W) % TPL, b = threadIdx.x / (W * TPL);
    const int tile = (int)(blk % a.ntx), z = (int)(blk / a.ntx) * B + b;
    const int kx = tile * W + c;
    const bool act = kx < a.H && z < N;
    // FP32: the twiddles first (where the line allows), so that no stage of
    // the transform waits for a table load after the data have arrived (5%
    // faster FP32 y passes at 512^3; FP64 measured no gain, its y passes a
    // little slower, and neither precision's z pass gained)
    constexpr bool YPRE = sizeof(T) == 4 && TwPre<T, N>::OK;
    TwPre<T, N> pre;
    if constexpr (YPRE) twiddle_preload(pre, a.tw, t, 1);
    // planes past the last (ragged workgroups of small grids) are clamped so
    // that the loads, issued unconditionally to be in flight together, stay
    // in bounds; only act lanes store
    cx<T> *g = a.Q + (long)(z < N ? z : 0) * a.PZ + kx;
    cx<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const cx<T> x = g[(long)(t + j * TPL) * a.P];
        v[j] = x;
    }
    fft_line<T, N, DIR>(v, lds + c + W * b, W * B, t, a.tw, 1,
                        YPRE ? &pre : nullptr);
    if (act) {
#pragma unroll
        for (int j = 0; j < E; ++j) g[(long)(t + j * TPL) * a.P] = v[j];
    }
}

template <typename T, int N, int W, int DIR>
__global__ __launch_bounds__((YZCfg<N, W>::NT)) void k_ypass(YArgs<T> a)
{
    using C = YZCfg<N, W>;
    __shared__ cx<T> lds[W * C::B * lslots<N>()];
    if (a.ctl && a.ctl->flag) return;
    ybody<T, N, W, DIR>(a, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// z pass: c2c along z, with the eq. (2) update on the hot path
// ---------------------------------------------------------------------------

enum ZMode {
    Z_STEP = 0,       // forward z, update, energy, store v^{n+1}, inverse z of v^{n+1}/M
    Z_FWD_STATE = 1,  // forward z -> state buffer
    Z_FWD_Q = 2,      // forward z in place
    Z_INV_STATE = 3,  // state buffer * scale -> inverse z -> Q
    Z_INV_Q = 4,      // inverse z in place, times scale
    Z_START = 5,      // symmetric start: Sp = (alpha/2) Sc - dt Fz(Q) + (beta/2) chi Sp
    Z_PAIR = 6        // energy partial of the stored pair (Sp = v^{-1}, Sc = v^0), no transform
};

// Time levels.  FP64 keeps two levels, v^n and v^{n-1} (Sp holds v^{n-1} and
// receives v^{n+1}).  FP32 stores the increment form v^n (Sc) and
// Delta^n = v^n - v^{n-1} (Sp), both updated in place, with the update done in
// FP64: rounding a stored pair of nearly equal FP32 levels would amplify by
// about 1/(omega dt), rounding their difference does not.
template <typename T>
constexpr bool increment_form() { return sizeof(T) == 4; }

template <typename T>
struct ZArgs {
    cx<T> *Q;
    const cx<T> *tw;
    cx<T> *Sp;        // Z_STEP: v^{n-1} (FP64) or Delta^n (FP32), updated; Z_FWD_STATE: output;
                      // Z_START: N^0 in, v^{-1} (FP64) or Delta^0 (FP32) out
    cx<T> *Sc;        // Z_STEP / Z_START: v^n (updated in place for FP32); Z_INV_STATE: input
    const cx<T> *Ssub;  // Z_INV_STATE: if set, the input is Sc - Ssub
    double *part;     // Z_STEP: energy partial per workgroup
    const Ctl *ctl;
    int P, H, ntx;
    long PZ;
    double ks2;       // (2 pi / L)^2
    double dt;
    double chi;
    double scale;     // 1/M for Z_STEP and Z_INV_STATE
    int has_vel;      // Z_START: Q holds F_xy[u_t0]
    int cf;           // complex field: kx runs over 0..N-1 (signed wavenumbers), every
                      // mode has energy weight 1
    int dkc;          // > 0: 2/3-rule dealiasing, the nonlinear term keeps the modes with
                      // |m| <= dkc (= N/3) on every axis; 0: no truncation
};

// Signed mode number of index k on an axis of N points.
template <int N>
__device__ __forceinline__ int mode_of(int k) { return k <= N / 2 ? k : k - N; }

// Largest |m| of the modes the nonlinear term keeps: dkc when dealiasing,
// else N (every mode).
template <int N>
__device__ __forceinline__ int keep_cut(int dkc) { return dkc > 0 ? dkc : N; }

// Energy weight of column kx: the half spectrum of a real field stands for
// the full one (kx and N - kx), except on the kx = 0 and kx = N/2 planes.
template <int N>
__device__ __forceinline__ double kx_weight(int kx, int cf)
{
    return (cf || kx == 0 || kx == N / 2) ? 1.0 : 2.0;
}

// alpha, beta of eq. (2) and omega^2 for mode numbers (mx, my, mz).
__device__ __forceinline__ void coeffs(int mx, int my, int mz, double ks2, double dt, double &al,
                                       double &be, double &w2)
{
    w2 = 1.0 + ks2 * (double)(mx * mx + my * my + mz * mz);
    const double a = 0.25 * w2 * dt * dt;
    const double inv = 1.0 / (1.0 + a);
    al = 2.0 * (1.0 - a) * inv;
    be = dt * dt * inv;
}

// The eq. (2) update of one mode (mx, my, mz) in FP64 from the stored levels
// vc = v^n and vp (v^{n-1}, or Delta^n in the increment form) and the
// transformed nonlinear term nl: nv = v^{n+1} and, in the increment form,
// nd = Delta^{n+1} = Delta^n - (2 - alpha) v^n + beta N^n, both rounded to T
// once.  Adds wgt times the mode's linear energy of (v^n, v^{n+1}) to esum
// (wgt = 0: a padding column, nothing added).
template <typename T>
__device__ __forceinline__ void zupdate(int mx, int my, int mz, double ks2, double dt, cx<T> vc,
                                        cx<T> vp, cx<T> nl, double wgt, double idt2, cx<T> &nv,
                                        cx<T> &nd, double &esum)
{
    double al, be, w2;
    coeffs(mx, my, mz, ks2, dt, al, be, w2);
    double nr, ni, dr, di;  // v^{n+1} and v^{n+1} - v^n in FP64
    if constexpr (increment_form<T>()) {
        const double c2 = 2.0 - al;
        dr = (double)vp.re - c2 * (double)vc.re + be * (double)nl.re;
        di = (double)vp.im - c2 * (double)vc.im + be * (double)nl.im;
        nr = (double)vc.re + dr;
        ni = (double)vc.im + di;
    } else {
        nr = al * (double)vc.re - (double)vp.re + be * (double)nl.re;
        ni = al * (double)vc.im - (double)vp.im + be * (double)nl.im;
        dr = nr - (double)vc.re;
        di = ni - (double)vc.im;
    }
    nv = mk((T)nr, (T)ni);
    nd = mk((T)dr, (T)di);
    if (wgt != 0.0) {
        const double sr = nr + (double)vc.re, sim = ni + (double)vc.im;
        esum += wgt * ((dr * dr + di * di) * idt2 + 0.25 * w2 * (sr * sr + sim * sim));
    }
    // the sum is formed here, mode by mode: left to the scheduler, the
    // additions (whose order is fixed) sink past the inverse transform and
    // keep every mode's term live in the meantime
    asm volatile("" : "+v"(esum));
}

// One workgroup's tile of the z pass: columns tile*W.. of B consecutive ky.
template <typename T, int N, int W, int MODE>
__device__ __forceinline__ void zbody(const ZArgs<T> &a, long blk, cx<T> *lds, double *part)
{
    using C = YZCfg<N, W>;
    constexpr int E = Radix<N>::E, TPL = C::TPL, B = C::B, NT = C::NT;
    const int c = threadIdx.x % W, t = (threadIdx.x / W) % TPL, b = threadIdx.x / (W * TPL);
    const int tile = (int)(blk % a.ntx), ky = (int)(blk / a.ntx) * B + b;
    const int kx = tile * W + c;
    const bool act = kx < a.H && ky < N;
    const long zs = a.PZ;
    // rows past the last ky (ragged workgroups of small grids) are clamped so
    // that every address formed stays in bounds (the state loads are
    // unconditional); only act lanes store
    cx<T> *g = a.Q + (long)(ky < N ? ky : 0) * a.P + kx;
    const long sbase = (((long)(ky < N ? ky : 0) * a.ntx + tile) * N) * W + c;
    cx<T> *lline = lds + c + W * b;
    const cx<T> zero = mk<T>(0, 0);
    cx<T> v[E];

    if constexpr (MODE == Z_PAIR) {
        double esum = 0.0;
        if (act) {
            const int my = ky <= N / 2 ? ky : ky - N, mxx = mode_of<N>(kx);
            const double wgt = kx_weight<N>(kx, a.cf);
            const double idt2 = 1.0 / (a.dt * a.dt);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int kz = t + j * TPL, mz = kz <= N / 2 ? kz : kz - N;
                double al, be, w2;
                coeffs(mxx, my, mz, a.ks2, a.dt, al, be, w2);
                const long si = sbase + (long)kz * W;
                const cx<T> a0 = a.Sp[si], a1 = a.Sc[si];
                double dr, di, sr, sim;
                if constexpr (increment_form<T>()) {  // Sc = v^0, Sp = Delta^0
                    dr = (double)a0.re;
                    di = (double)a0.im;
                    sr = 2.0 * (double)a1.re - dr;
                    sim = 2.0 * (double)a1.im - di;
                } else {
                    dr = (double)a1.re - (double)a0.re;
                    di = (double)a1.im - (double)a0.im;
                    sr = (double)a1.re + (double)a0.re;
                    sim = (double)a1.im + (double)a0.im;
                }
                esum += wgt * ((dr * dr + di * di) * idt2 + 0.25 * w2 * (sr * sr + sim * sim));
            }
        }
        block_max_sum<NT>(0.0, esum, part);
        return;
    }
    if constexpr (MODE == Z_STEP || MODE == Z_FWD_STATE || MODE == Z_FWD_Q || MODE == Z_START) {
        if (MODE != Z_START || a.has_vel) {
            // padding columns (kx >= H, allocated) are loaded and transformed
            // like the others; nothing they produce is stored or summed
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = ld_nt(g + (t + j * TPL) * zs);
            fft_line<T, N, -1>(v, lline, W * B, t, a.tw, 1);
        } else {
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = zero;
        }
    }
    if constexpr (MODE == Z_FWD_Q) {
        if (act) {
#pragma unroll
            for (int j = 0; j < E; ++j) g[(t + j * TPL) * zs] = v[j];
        }
        return;
    }
    if constexpr (MODE == Z_FWD_STATE) {
        if (act) {
#pragma unroll
            for (int j = 0; j < E; ++j) a.Sp[sbase + (long)(t + j * TPL) * W] = v[j];
        }
        return;
    }
    const int my = ky <= N / 2 ? ky : ky - N, mxx = mode_of<N>(kx);
    // dealiasing: the (x, y) part of the kept-mode test, per lane
    const int kcut = keep_cut<N>(a.dkc);
    const bool keep_xy = abs(mxx) <= kcut && abs(my) <= kcut;
    if constexpr (MODE == Z_START) {
        if (act) {
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int kz = t + j * TPL, mz = kz <= N / 2 ? kz : kz - N;
                double al, be, w2;
                coeffs(mxx, my, mz, a.ks2, a.dt, al, be, w2);
                const long si = sbase + (long)kz * W;
                const cx<T> vc = a.Sc[si];
                const cx<T> nl = keep(a.chi != 0.0 && keep_xy && abs(mz) <= kcut, a.Sp[si]);
                double re, im;
                if constexpr (increment_form<T>()) {
                    // Delta^0 = v^0 - v^{-1} = (2a/(1+a)) v^0 + dt F[u_t0] - (beta/2) chi N^0
                    const double c0 = 1.0 - 0.5 * al;  // = 2a/(1+a), no cancellation for small a
                    re = c0 * (double)vc.re + a.dt * (double)v[j].re - 0.5 * be * a.chi * (double)nl.re;
                    im = c0 * (double)vc.im + a.dt * (double)v[j].im - 0.5 * be * a.chi * (double)nl.im;
                } else {
                    re = 0.5 * al * (double)vc.re - a.dt * (double)v[j].re +
                         0.5 * be * a.chi * (double)nl.re;
                    im = 0.5 * al * (double)vc.im - a.dt * (double)v[j].im +
                         0.5 * be * a.chi * (double)nl.im;
                }
                a.Sp[si] = mk((T)re, (T)im);
            }
        }
        return;
    }
    double esum = 0.0;
    if constexpr (MODE == Z_STEP) {
        const double wgt = kx_weight<N>(kx, a.cf);
        const double idt2 = 1.0 / (a.dt * a.dt);
        // The state loads of a batch of ZB positions are issued before any is
        // used, unconditionally (the padding columns of the last tile are
        // allocated), so they are in flight together; loads under a
        // per-position branch would each wait for their own data before the
        // next is issued.  FP64 batches 4 positions to stay within 128 VGPRs
        // (1, 2 and 8 measured slower at 512^3); FP32 takes 8, or 6 for the
        // 12 positions of 3 * 2^a sizes (12 at once spill registers).
        constexpr int ZB0 = sizeof(T) == 8 ? 4 : 8;
        constexpr int ZB = E % ZB0 == 0 ? ZB0 : E % 6 == 0 && ZB0 >= 6 ? 6 : E % 4 == 0 ? 4 : E;
        static_assert(E % ZB == 0, "state-load batches must tile the positions");
#pragma unroll
        for (int h = 0; h < E / ZB; ++h) {
          cx<T> vcs[ZB], vps[ZB];
#pragma unroll
          for (int i = 0; i < ZB; ++i) {
              const long si = sbase + (long)(t + (h * ZB + i) * TPL) * W;
              vcs[i] = ld_nt(a.Sc + si);
              vps[i] = ld_nt(a.Sp + si);
          }
#pragma unroll
          for (int i = 0; i < ZB; ++i) {
            const int j = h * ZB + i;
            const int kz = t + j * TPL, mz = kz <= N / 2 ? kz : kz - N;
            const long si = sbase + (long)kz * W;
            const cx<T> nl = keep(keep_xy && abs(mz) <= kcut, v[j]);
            cx<T> nv, nd;
            zupdate(mxx, my, mz, a.ks2, a.dt, vcs[i], vps[i], nl, act ? wgt : 0.0, idt2, nv, nd, esum);
            if (act) {
                if constexpr (increment_form<T>()) {
                    st_nt(a.Sc + si, nv);
                    st_nt(a.Sp + si, nd);
                } else {
                    st_nt(a.Sp + si, nv);
                }
            }
            // the stored level, scaled as a resumed run scales it (Z_INV_STATE)
            v[j] = scale(nv, (T)a.scale);
          }
        }
        __syncthreads();
    } else if constexpr (MODE == Z_INV_STATE) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const long si = sbase + (long)(t + j * TPL) * W;
            if (act && a.Ssub) {
                const cx<T> x = a.Sc[si], y = a.Ssub[si];
                v[j] = mk((T)(((double)x.re - (double)y.re) * a.scale),
                          (T)(((double)x.im - (double)y.im) * a.scale));
            } else {
                v[j] = scale(a.Sc[si], (T)a.scale);
            }
        }
    } else if constexpr (MODE == Z_INV_Q) {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = scale(g[(t + j * TPL) * zs], (T)a.scale);
        __syncthreads();
    }
    // Recompute the inverse transform's LDS addresses and the store addresses
    // here rather than keep those of the forward transform and the loads live
    // (an empty asm hides the earlier values of t and of g's offset from the
    // compiler; g itself stays a global pointer, so the stores stay global
    // rather than flat ones).
    int ti = t;
    long go = g - a.Q;
    asm volatile("" : "+v"(ti), "+v"(go));
    cx<T> *gi = a.Q + go;
    fft_line<T, N, 1>(v, lline, W * B, ti, a.tw, 1);
    if (act) {
#pragma unroll
        for (int j = 0; j < E; ++j) st_nt(gi + (ti + j * TPL) * zs, v[j]);
    }
    if constexpr (MODE == Z_STEP) block_max_sum<NT>(0.0, esum, part);
}

// Waves per SIMD that the LDS of a z-pass workgroup allows (160 KiB per CU,
// 4 SIMDs); asking the compiler for that occupancy keeps the register count
// from being the tighter limit.  FP32 stays at 4: the 1024-thread FP32 tiles
// would need 8 (64 VGPRs, with spills) and ran slower that way, as did
// 512-thread tiles of 16 values per thread (measured at 512^3).
template <typename T, int N, int W>
constexpr int z_waves()
{
    using C = YZCfg<N, W>;
    constexpr long lds = (long)sizeof(cx<T>) * W * C::B * lslots<N>() + 256;
    constexpr int wg = (int)(163840 / lds);
    constexpr int w = wg * (C::NT / 64) / 4;
    constexpr int cap = sizeof(T) == 8 ? 8 : 4;
    return w < 1 ? 1 : w > cap ? cap : w;
}

template <typename T, int N, int W, int MODE>
__global__ __launch_bounds__((YZCfg<N, W>::NT)) __attribute__((amdgpu_waves_per_eu(z_waves<T, N, W>())))
void k_zpass(ZArgs<T> a)
{
    using C = YZCfg<N, W>;
    __shared__ cx<T> lds[W * C::B * lslots<N>()];
    if constexpr (MODE == Z_STEP) {
        if (a.ctl->flag) return;
    }
    zbody<T, N, W, MODE>(a, blockIdx.x, lds, a.part + 2 * blockIdx.x);
}

// The z pass of a step (Z_STEP) as a persistent, software-pipelined kernel:
// workgroup g takes the tiles g, g + G, g + 2G, ... (G = gridDim.x, about
// one workgroup per CU) and keeps the next tile's loads in flight while it
// transforms the current one:
//   top:     PF = 1: the current tile's Q values arrive (issued one tile
//            earlier) and the next tile's Q loads are issued; PF = 0: the
//            current tile's Q loads are issued and arrive;
//   forward z transform; the state loads (issued one tile earlier) arrive;
//   update, energy term, state stores; the next tile's state loads issued;
//   inverse z transform; Q stores.
// Loads complete in issue order (one counter per wave), so every wait above
// leaves the loads issued after it in flight; the twiddle table is copied to
// LDS first so that no table load is queued behind the prefetches.  Each
// workgroup sums its energy terms in its fixed tile order and writes one
// partial, G partials in all.  The values stored are those of k_zpass's
// Z_STEP (same transforms, same update).
template <typename T, int N, int W, int PF>
__global__ __launch_bounds__((YZCfg<N, W>::NT)) void k_zstep(ZArgs<T> a, int nblk)
{
    using C = YZCfg<N, W>;
    constexpr int E = Radix<N>::E, TPL = C::TPL, B = C::B, NT = C::NT;
    __shared__ cx<T> lds[W * B * lslots<N>()];
    __shared__ cx<T> twl[N];
    if (a.ctl->flag) return;
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = a.tw[i];
    const double idt2 = 1.0 / (a.dt * a.dt);
    const int kcut = keep_cut<N>(a.dkc);
    double esum = 0.0;
    // This thread's place in a tile, (column c, position t, row b), read
    // through an empty asm wherever addresses are formed: the compiler then
    // rebuilds them in each tile instead of hoisting every loop-invariant
    // offset (some hundred registers) out of the tile loop.
    struct Lane {
        int c, t, b;
    };
    auto lane = []() {
        Lane l{(int)threadIdx.x % W, ((int)threadIdx.x / W) % TPL, (int)threadIdx.x / (W * TPL)};
        asm volatile("" : "+v"(l.c), "+v"(l.t), "+v"(l.b));
        return l;
    };
    // Q and state addresses of tile blk; rows past the last ky (ragged
    // workgroups of small grids) are clamped, so every load is
    // unconditional and in bounds (padding columns are allocated)
    auto qptr = [&](int blk, const Lane &l) -> cx<T> * {
        const int ky = (blk / a.ntx) * B + l.b;
        return a.Q + (long)(ky < N ? ky : 0) * a.P + (blk % a.ntx) * W + l.c + (long)l.t * a.PZ;
    };
    auto sptr = [&](cx<T> *S, int blk, const Lane &l) -> cx<T> * {
        const int ky = (blk / a.ntx) * B + l.b;
        return S + (((long)(ky < N ? ky : 0) * a.ntx + blk % a.ntx) * N + l.t) * W + l.c;
    };
    auto load_q = [&](cx<T> (&q)[E], int blk) {
        const Lane l = lane();
        const cx<T> *g = qptr(blk, l);
#pragma unroll
        for (int j = 0; j < E; ++j) q[j] = ld_nt(g + (long)j * TPL * a.PZ);
    };
    auto load_s = [&](cx<T> (&sc)[E], cx<T> (&sp)[E], int blk) {
        const Lane l = lane();
        const cx<T> *gc = sptr(a.Sc, blk, l), *gp = sptr(a.Sp, blk, l);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            sc[j] = ld_nt(gc + j * TPL * W);
            sp[j] = ld_nt(gp + j * TPL * W);
        }
    };
    cx<T> q[E], sc[E], sp[E];
    if constexpr (PF == 1) load_q(q, blockIdx.x);
    load_s(sc, sp, blockIdx.x);
    __syncthreads();  // twiddles in LDS
    for (int it = blockIdx.x; it < nblk; it += gridDim.x) {
        int blk = it;
        asm volatile("" : "+s"(blk));
        const int nxt = blk + gridDim.x;
        cx<T> v[E];
        if constexpr (PF == 1) {
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = q[j];
            if (nxt < nblk) load_q(q, nxt);
        } else {
            load_q(v, blk);
        }
        Lane l = lane();
        const int ky = (blk / a.ntx) * B + l.b, kx = (blk % a.ntx) * W + l.c;
        const bool act = kx < a.H && ky < N;
        fft_line<T, N, -1>(v, lds + l.c + W * l.b, W * B, l.t, twl, 1);
        l = lane();
        const int my = ky <= N / 2 ? ky : ky - N, mxx = mode_of<N>(kx);
        const bool keep_xy = abs(mxx) <= kcut && abs(my) <= kcut;
        const double wgt = act ? kx_weight<N>(kx, a.cf) : 0.0;
        cx<T> *gc = sptr(a.Sc, blk, l), *gp = sptr(a.Sp, blk, l);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int kz = l.t + j * TPL, mz = kz <= N / 2 ? kz : kz - N;
            const cx<T> nl = keep(keep_xy && abs(mz) <= kcut, v[j]);
            cx<T> nv, nd;
            zupdate(mxx, my, mz, a.ks2, a.dt, sc[j], sp[j], nl, wgt, idt2, nv, nd, esum);
            if (act) {
                if constexpr (increment_form<T>()) {
                    st_nt(gc + j * TPL * W, nv);
                    st_nt(gp + j * TPL * W, nd);
                } else {
                    st_nt(gp + j * TPL * W, nv);
                }
            }
            v[j] = scale(nv, (T)a.scale);
        }
        if (nxt < nblk) load_s(sc, sp, nxt);
        __syncthreads();
        l = lane();
        fft_line<T, N, 1>(v, lds + l.c + W * l.b, W * B, l.t, twl, 1);
        if (act) {
            cx<T> *g = qptr(blk, l);
#pragma unroll
            for (int j = 0; j < E; ++j) st_nt(g + (long)j * TPL * a.PZ, v[j]);
        }
        __syncthreads();  // the next tile's forward transform reuses the LDS
    }
    block_max_sum<NT>(0.0, esum, a.part + 2 * blockIdx.x);
}

// Linear energy partials of a pair of levels stored in the state layout:
// sum w_k [|v1 - v0|^2/dt^2 + omega_k^2 |v1 + v0|^2 / 4] (w_k = 1 on the kx = 0
// and kx = n/2 planes, 2 elsewhere: the half spectrum stands for the full one;
// w_k = 1 throughout for a complex field, cf).
// S0 = v^{-1}, S1 = v^0 for two levels; S0 = v^0, S1 = Delta^0 for the
// increment form.
template <typename T, int N, int W>
__global__ __launch_bounds__(256) void k_pair_energy(const cx<T> *S0, const cx<T> *S1, double *part,
                                                     int H, int ntx, double ks2, double dt, int cf)
{
    const long total = (long)N * ntx * N * W;
    double esum = 0.0;
    const double idt2 = 1.0 / (dt * dt);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const int c = (int)(i % W);
        const int kz = (int)((i / W) % N);
        const long rest = i / ((long)W * N);
        const int tile = (int)(rest % ntx), ky = (int)(rest / ntx);
        const int kx = tile * W + c;
        if (kx >= H) continue;
        const int my = ky <= N / 2 ? ky : ky - N, mz = kz <= N / 2 ? kz : kz - N;
        double al, be, w2;
        coeffs(mode_of<N>(kx), my, mz, ks2, dt, al, be, w2);
        const double wgt = kx_weight<N>(kx, cf);
        const cx<T> a0 = S0[i], a1 = S1[i];
        double dr, di, sr, si;
        if constexpr (increment_form<T>()) {
            dr = (double)a1.re;
            di = (double)a1.im;
            sr = 2.0 * (double)a0.re - dr;
            si = 2.0 * (double)a0.im - di;
        } else {
            dr = (double)a1.re - (double)a0.re;
            di = (double)a1.im - (double)a0.im;
            sr = (double)a1.re + (double)a0.re;
            si = (double)a1.im + (double)a0.im;
        }
        esum += wgt * ((dr * dr + di * di) * idt2 + 0.25 * w2 * (sr * sr + si * si));
    }
    block_max_sum<256>(0.0, esum, part + 2 * blockIdx.x);
}

// Gather a state-layout level (S, or S - Ssub when Ssub is set) into the
// half-spectrum layout [kz][ky][kx] (pitch H) of doubles.
template <typename T, int N, int W>
__global__ __launch_bounds__(256) void k_state_to_spec(const cx<T> *S, const cx<T> *Ssub, double *out,
                                                       int H, int ntx)
{
    const long total = (long)N * N * H;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const int kx = (int)(i % H);
        const int ky = (int)((i / H) % N);
        const int kz = (int)(i / ((long)H * N));
        const long si = (((long)ky * ntx + kx / W) * N + kz) * W + (kx % W);
        double re = (double)S[si].re, im = (double)S[si].im;
        if (Ssub) {
            re -= (double)Ssub[si].re;
            im -= (double)Ssub[si].im;
        }
        out[2 * i] = re;
        out[2 * i + 1] = im;
    }
}

// Working field Q (row pitch P, plane pitch PZ, n rows per plane) <-> half
// spectrum of doubles (pitch H).
template <typename T>
__global__ __launch_bounds__(256) void k_q_to_spec(const cx<T> *Q, double *out, int P, long PZ, int n,
                                                   int H, long rows)
{
    const long total = rows * H;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long r = i / H;
        const int k = (int)(i % H);
        const cx<T> v = Q[(r / n) * PZ + (r % n) * P + k];
        out[2 * i] = (double)v.re;
        out[2 * i + 1] = (double)v.im;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_spec_to_q(const double *in, cx<T> *Q, int P, long PZ, int n,
                                                   int H, long rows)
{
    const long total = rows * P;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long r = i / P;
        const int k = (int)(i % P);
        Q[(r / n) * PZ + (r % n) * P + k] =
            k < H ? mk((T)in[2 * (r * H + k)], (T)in[2 * (r * H + k) + 1]) : mk<T>(0, 0);
    }
}

// Fixed-order reduction of the workgroup partials, in two launches so that
// many workgroups share the reading: k_reduce_partials folds contiguous slices
// of the x-pass partials (max, sum) and z-pass partials (sum) into RSUB
// sub-partials, then k_finalize folds those.  Both use fixed index orders, so
// the result is bitwise reproducible.
constexpr int RSUB = 128;

static __global__ __launch_bounds__(256) void k_reduce_partials(const double *partA, int nA,
                                                         const double *partC, int nC, double *sub,
                                                         const Ctl *ctl, int check_flag)
{
    if (check_flag && ctl->flag) return;
    const int b = blockIdx.x;
    const int a0 = (int)((long)nA * b / RSUB), a1 = (int)((long)nA * (b + 1) / RSUB);
    const int c0 = (int)((long)nC * b / RSUB), c1 = (int)((long)nC * (b + 1) / RSUB);
    double mx = 0.0, s4 = 0.0, se = 0.0;
    for (int i = a0 + (int)threadIdx.x; i < a1; i += 256) {
        mx = nanmax(mx, partA[2 * i]);
        s4 += partA[2 * i + 1];
    }
    for (int i = c0 + (int)threadIdx.x; i < c1; i += 256) se += partC[2 * i + 1];
    __shared__ double red[3][256];
    red[0][threadIdx.x] = mx;
    red[1][threadIdx.x] = s4;
    red[2][threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = nanmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sub[3 * b] = red[0][0];
        sub[3 * b + 1] = red[1][0];
        sub[3 * b + 2] = red[2][0];
    }
}

//   mode 0 (step):   rec[step] = {elin, q4, maxu}; blow-up test; energy
//                    alarm; step counter.
//   mode 1 (reduce): rec[step].q4/maxu from the x-pass partials only.
//   mode 2 (init):   ctl->elin_m, q4_m, maxu_m.
// The energy alarm follows the paper's use of the conserved energy (Sec. 1.1)
// as a check on the code and the machine: at level n the step has everything
// for E^{n-1/2} = elin(v^{n-1}, v^n) - chi (Q4^{n-1} + Q4^n)/8, evaluated in
// the same order as the host's energy series, so the alarm and kg_energies
// see the same value.  The first step stores E^{-1/2} as the reference.
static __global__ __launch_bounds__(RSUB) void k_finalize(const double *sub, Rec *rec, Ctl *ctl,
                                                   double thr, double escale, double h3,
                                                   double chi, int mode)
{
    if (mode != 2 && ctl->flag) return;
    __shared__ double red[3][RSUB];
    red[0][threadIdx.x] = sub[3 * threadIdx.x];
    red[1][threadIdx.x] = sub[3 * threadIdx.x + 1];
    red[2][threadIdx.x] = mode == 1 ? 0.0 : sub[3 * threadIdx.x + 2];
    __syncthreads();
    for (int s = RSUB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = nanmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double maxu = red[0][0], q4 = h3 * red[1][0], elin = escale * red[2][0];
    const bool bad = !(maxu <= 1.7976931348623157e308);  // NaN or inf
    if (mode == 2) {
        ctl->elin_m = elin;
        ctl->q4_m = q4;
        ctl->maxu_m = bad ? __builtin_nan("") : maxu;
        return;
    }
    const int n = ctl->step;
    Rec *r = rec + (n & (RING - 1));
    r->q4 = q4;
    r->maxu = bad ? __builtin_nan("") : maxu;
    if (mode == 1) return;
    r->elin = elin;
    if (bad || (thr > 0.0 && maxu > thr)) {
        ctl->flag = 1;
        ctl->blow_step = n;
        return;
    }
    const Rec *rp = rec + ((n - 1) & (RING - 1));
    const double ep = n == 0 ? ctl->elin_m : rp->elin;
    const double qp = n == 0 ? ctl->q4_m : rp->q4;
    const double E = ep - chi * (qp + q4) / 8.0;
    if (n == 0) {
        ctl->e_ref = E;
    } else if (ctl->e_tol > 0.0 && !(fabs(E - ctl->e_ref) <= ctl->e_tol * fabs(ctl->e_ref))) {
        ctl->flag = 2;  // a non-finite energy trips it too
        ctl->blow_step = n;
        return;
    }
    ctl->step = n + 1;
}

// Plain copy (bandwidth ceiling and counter calibration): every byte read and
// written once, four 16-byte values in flight per thread, streaming hints.
static __global__ __launch_bounds__(256) void k_copy(uint4 *dst, const uint4 *src, long n16)
{
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const long stride = (long)gridDim.x * 256 * 4;
    for (long b = (long)blockIdx.x * 256 * 4 + threadIdx.x; b < n16; b += stride) {
        v4u r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long i = b + (long)u * 256;
            if (i < n16) r[u] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(src) + i);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long i = b + (long)u * 256;
            if (i < n16) __builtin_nontemporal_store(r[u], reinterpret_cast<v4u *>(dst) + i);
        }
    }
}

}  // namespace kg
