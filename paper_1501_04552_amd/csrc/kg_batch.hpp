// kg_batch.hpp -- persistent kernels of the batched parametric sweep.
//
// Many independent runs of eq. (2) (Sec. 1.1.2), each with its own grid size
// and Gaussian initial data, advance together: every pass of a step is one
// persistent launch whose workgroups stride over the (run, tile) tasks of
// all active runs, whatever their sizes.  Runs retire independently on
// blow-up or at their last step; their tasks are then skipped.  The pass
// bodies are those of the single-run kernels.  The sweep serves the paper's
// motivation of parametric blow-up studies without symmetry assumptions
// (Sec. 1).
#pragma once

#include "kg_kernels.hpp"

namespace kg {

// Device run table entry.
struct BRun {
    int n, H, P, ntx, W;
    int flag;  // 0 active, 1 blown up, 2 finished (max_steps reached)
    int step, max_steps, blow_step;
    int xoff, nxt, zoff, nzt;  // partial slots of the run's x and z tasks
    double dt, ks2, invM, escale, h3, chi, thr;
    double A, sx, sy, sz, L;
    double elin_m, q4_m;              // linear energy of (v^{-1}, v^0) and Q4^{-1}
    double E0;                        // E^{-1/2}
    double elin_last, q4_prev, q4_cur;  // newest pair / levels
    double maxu_max;                  // max over levels of max|u|
    double E_final;
    void *Q, *S0, *S1;
    const void *tw;
};

struct BTask {
    int run;
    int blk;
};

// Task list in device memory, so captured graphs stay valid when it shrinks.
struct BList {
    BTask *tasks;
    int *count;
};

template <typename T>
__device__ __forceinline__ XArgs<T> x_args(const BRun &R, double *part)
{
    XArgs<T> a{};
    a.Q = (cx<T> *)R.Q;
    a.tw = (const cx<T> *)R.tw;
    a.part = part;
    a.P = R.P;
    a.PZ = (long)R.n * R.P;
    a.chi = (T)R.chi;
    a.gA = R.A;
    a.gsx = R.sx;
    a.gsy = R.sy;
    a.gsz = R.sz;
    a.gL = R.L;
    return a;
}

template <typename T>
__device__ __forceinline__ YArgs<T> y_args(const BRun &R)
{
    YArgs<T> a{};
    a.Q = (cx<T> *)R.Q;
    a.tw = (const cx<T> *)R.tw;
    a.P = R.P;
    a.PZ = (long)R.n * R.P;
    a.H = R.H;
    a.ntx = R.ntx;
    return a;
}

// ZArgs of a run.  sel picks the time-level buffers:
//   0: step (Sc = v^m, Sp = v^{m-1} by the parity of the run's step m)
//   1: Sp = S1 (init outputs into S1);  2: Sp = S0;  3: Sc = S1 (inverse of v^{-1});
//   4: Sc = S0 (inverse of v^0), 5: start (Sp = S1, Sc = S0).
template <typename T>
__device__ __forceinline__ ZArgs<T> z_args(const BRun &R, int sel, double *part)
{
    ZArgs<T> a{};
    a.Q = (cx<T> *)R.Q;
    a.tw = (const cx<T> *)R.tw;
    a.part = part;
    a.P = R.P;
    a.PZ = (long)R.n * R.P;
    a.H = R.H;
    a.ntx = R.ntx;
    a.ks2 = R.ks2;
    a.dt = R.dt;
    a.chi = R.chi;
    a.scale = R.invM;
    cx<T> *S0 = (cx<T> *)R.S0, *S1 = (cx<T> *)R.S1;
    switch (sel) {
    case 0:
        a.Sc = (R.step & 1) ? S1 : S0;
        a.Sp = (R.step & 1) ? S0 : S1;
        break;
    case 1: a.Sp = S1; break;
    case 2: a.Sp = S0; break;
    case 3: a.Sc = S1; break;
    case 4: a.Sc = S0; break;
    case 5:
        a.Sp = S1;
        a.Sc = S0;
        break;
    }
    return a;
}

// Persistent passes over the tasks of all runs of one grid size N (one
// kernel per size keeps each size's register and LDS budget its own); the
// sizes of a sweep run as concurrent branches of one graph.  Waves per SIMD
// requested per size: as many as the LDS allows without register spills
// (measured with the compiler's resource report).
template <int N>
constexpr int batch_waves() { return N == 64 ? 4 : N == 128 ? 3 : 2; }
template <typename T, int N, int MODE>
__global__ __launch_bounds__(256, batch_waves<N>()) void kb_xpass(BRun *runs, BList L, double *part, int want, int cube)
{
    static_assert(XCfg<T, N>::NT == 256, "batch workgroups have 256 threads");
    __shared__ cx<T> rows[XCfg<T, N>::PPB * XCfg<T, N>::RS];
    const int cnt = *L.count;
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const BTask tk = L.tasks[i];
        const BRun &R = runs[tk.run];
        if (R.flag != want) continue;
        XArgs<T> a = x_args<T>(R, part + 2 * i);
        if (MODE == X_GAUSS) a.chi = cube ? (T)1 : (T)0;  // cube the sampled data or not
        xbody<T, N, MODE>(a, tk.blk, rows, part + 2 * i);
        __syncthreads();  // the next task reuses the LDS
    }
}

template <typename T, int N, int W, int DIR>
__global__ __launch_bounds__(256) void kb_ypass(BRun *runs, BList L, int want)
{
    static_assert(YZCfg<N, W>::NT == 256, "batch workgroups have 256 threads");
    __shared__ cx<T> lds[W * YZCfg<N, W>::B * lslots<N>()];
    const int cnt = *L.count;
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const BTask tk = L.tasks[i];
        const BRun &R = runs[tk.run];
        if (R.flag != want) continue;
        ybody<T, N, W, DIR>(y_args<T>(R), tk.blk, lds);
        __syncthreads();
    }
}

template <typename T, int N, int W, int MODE>
__global__ __launch_bounds__(256, batch_waves<N>()) void kb_zpass(BRun *runs, BList L, double *part, int want, int sel)
{
    static_assert(YZCfg<N, W>::NT == 256, "batch workgroups have 256 threads");
    __shared__ cx<T> lds[W * YZCfg<N, W>::B * lslots<N>()];
    const int cnt = *L.count;
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const BTask tk = L.tasks[i];
        const BRun &R = runs[tk.run];
        if (R.flag != want) continue;
        zbody<T, N, W, MODE>(z_args<T>(R, sel, part + 2 * i), tk.blk, lds, part + 2 * i);
        __syncthreads();
    }
}

// Per-run fixed-order reduction of the partials and the run's bookkeeping.
//   mode 0 (step):  record level m = step: max|u|, Q4^m, linear energy of
//                   (v^m, v^{m+1}); blow-up test; step counter; retire.
//   mode 1 (init):  elin_m, q4_m of the initial pair.
//   mode 2 (final): Q4 of the last level of a finished run -> E_final.
enum BFin { BF_STEP = 0, BF_INIT = 1, BF_FINAL = 2 };

// `list` holds the run indices of one size class; the partial offsets of its
// runs refer to that class's task lists.
__global__ __launch_bounds__(256) void kb_finalize(BRun *runs, const int *list, int nlist,
                                                   const double *partA, const double *partC, int mode,
                                                   int want)
{
    __shared__ double red[3][256];
    for (int q = blockIdx.x; q < nlist; q += gridDim.x) {
        BRun &R = runs[list[q]];
        if (R.flag != want) continue;
        double mx = 0.0, s4 = 0.0, se = 0.0;
        for (int i = threadIdx.x; i < R.nxt; i += 256) {
            mx = nanmax(mx, partA[2 * (R.xoff + i)]);
            s4 += partA[2 * (R.xoff + i) + 1];
        }
        if (mode != BF_FINAL)
            for (int i = threadIdx.x; i < R.nzt; i += 256) se += partC[2 * (R.zoff + i) + 1];
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
            const double maxu = red[0][0], q4 = R.h3 * red[1][0], elin = R.escale * red[2][0];
            const bool bad = !(maxu <= 1.7976931348623157e308);
            if (mode == BF_INIT) {
                R.elin_m = elin;
                R.q4_m = q4;
                R.maxu_max = 0.0;
            } else if (mode == BF_FINAL) {
                // the last level max_steps: its energy, and the blow-up test
                // every other level had (level 0 itself for zero-step runs)
                const int m = R.step;
                const double E = m == 0 ? R.elin_m - R.chi * (R.q4_m + q4) / 8.0
                                        : R.elin_last - R.chi * (R.q4_cur + q4) / 8.0;
                if (m == 0) R.E0 = E;
                R.E_final = E;
                R.maxu_max = nanmax(R.maxu_max, bad ? __builtin_nan("") : maxu);
                if (bad || (R.thr > 0.0 && maxu > R.thr)) {
                    R.flag = 1;
                    R.blow_step = m;
                }
            } else {
                const int m = R.step;
                if (m == 0) R.E0 = R.elin_m - R.chi * (R.q4_m + q4) / 8.0;
                R.maxu_max = nanmax(R.maxu_max, bad ? __builtin_nan("") : maxu);
                R.q4_prev = R.q4_cur;
                R.q4_cur = q4;
                R.elin_last = elin;
                if (bad || (R.thr > 0.0 && maxu > R.thr)) {
                    R.flag = 1;
                    R.blow_step = m;
                } else {
                    R.step = m + 1;
                    if (R.step >= R.max_steps) R.flag = 2;
                }
            }
        }
        __syncthreads();
    }
}

// Number of active runs (flag 0) into *active: one workgroup, read back by
// the host after each graph replay instead of the whole run table.
__global__ __launch_bounds__(256) void kb_count_active(const BRun *runs, int nruns, int *active)
{
    __shared__ int red[256];
    int c = 0;
    for (int r = threadIdx.x; r < nruns; r += 256) c += runs[r].flag == 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *active = red[0];
}

}  // namespace kg
