// kg_batch.hip -- host side of the batched parametric sweep (kg_batch_run).
//
// Runs of eq. (2) with Gaussian initial data and their own grid sizes advance
// together, each pass one persistent launch over the tiles of every active
// run; steps are replayed from a captured hipGraph.  Retired runs (blow-up or
// last step) drop out of the task lists between graph replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/kg.h"
#include "kg_batch.hpp"

using namespace kg;

namespace {

thread_local std::string g_err;

kg_status bfail(kg_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define BCHK(expr)                                                                 \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) return bfail(KG_E_HIP, std::string(#expr) + ": " +   \
                                                         hipGetErrorString(e_));   \
    } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool batch_size_ok(int n)
{
    return n == 32 || n == 48 || n == 64 || n == 96 || n == 128;
}

// Threads per line and outer lines per workgroup of the 256-thread bodies.
int tpl(int n) { return n % 3 == 0 ? n / 12 : n / 8; }
long x_tasks(int n) { return ((long)n * n / 2 + 256 / tpl(n) - 1) / (256 / tpl(n)); }
int yz_b(int n, int W)
{
    int b = 256 / (W * tpl(n));
    return b < 1 ? 1 : (b < n ? b : n);
}
long yz_tasks(int n, int W, int ntx) { return (long)ntx * ((n + yz_b(n, W) - 1) / yz_b(n, W)); }

// ---------------------------------------------------------------------------
// Tile-width cache: a flat JSON object {"fp64/48": 8, ...}
// ---------------------------------------------------------------------------

std::map<std::string, int> load_cache(const std::string &path)
{
    std::map<std::string, int> m;
    FILE *f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!f) return m;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        const size_t colon = s.find(':', end);
        if (colon == std::string::npos) break;
        m[key] = std::atoi(s.c_str() + colon + 1);
        pos = s.find_first_of(",}", colon);
        if (pos == std::string::npos) break;
    }
    return m;
}

void save_cache(const std::string &path, const std::map<std::string, int> &m)
{
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{");
    bool first = true;
    for (auto &kv : m) {
        std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    std::fprintf(f, "\n}\n");
    std::fclose(f);
}

std::string cache_key(int n) { return "fp64/" + std::to_string(n); }

// ---------------------------------------------------------------------------
// One batch
// ---------------------------------------------------------------------------

struct Batch {
    hipStream_t st = nullptr;
    int nruns = 0;
    std::vector<BRun> host;       // run table (host copy)
    std::vector<BTask> xfull, yfull;  // full task lists (run-major)
    std::vector<int> xoff0, zoff0;    // offsets of each run's tasks in the full lists
    void *arena = nullptr;
    BRun *d_runs = nullptr;
    BTask *d_xt = nullptr, *d_yt = nullptr;
    int *d_cnt = nullptr;  // [0] x tasks, [1] y/z tasks
    double *d_pa = nullptr, *d_pc = nullptr;
    int grid = 512;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    ~Batch()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cap) (void)hipStreamDestroy(cap);
        if (arena) (void)hipFree(arena);
    }
    BList xl() const { return BList{d_xt, d_cnt}; }
    BList yl() const { return BList{d_yt, d_cnt + 1}; }
};

kg_status setup(Batch &b, const kg_run_desc *runs, int nruns, const std::vector<int> &W, double L)
{
    b.nruns = nruns;
    b.host.assign(nruns, BRun{});
    // twiddle tables: one per distinct n
    std::map<int, size_t> tw_off;
    size_t off = 0;
    std::vector<size_t> qoff(nruns), s0off(nruns), s1off(nruns);
    for (int r = 0; r < nruns; ++r) {
        BRun &R = b.host[r];
        const kg_run_desc &d = runs[r];
        R.n = d.n;
        R.H = d.n / 2 + 1;
        R.W = W[r];
        R.ntx = (R.H + R.W - 1) / R.W;
        R.P = ((R.ntx * R.W + 7) / 8) * 8;
        R.flag = d.max_steps > 0 ? 0 : 2;
        R.step = 0;
        R.max_steps = d.max_steps;
        R.blow_step = -1;
        R.dt = d.dt;
        const double ks = 2.0 * M_PI / L;
        R.ks2 = ks * ks;
        const double M = (double)d.n * d.n * d.n, h = L / d.n;
        R.invM = 1.0 / M;
        R.h3 = h * h * h;
        R.escale = R.h3 / (2.0 * M);
        R.chi = 1.0;
        R.thr = d.threshold;
        R.A = d.A;
        R.sx = d.sx;
        R.sy = d.sy;
        R.sz = d.sz;
        R.L = L;
        R.E_final = std::nan("");
        const size_t q = up((size_t)d.n * d.n * R.P * 16);
        const size_t s = up((size_t)d.n * R.ntx * d.n * R.W * 16);
        qoff[r] = off;
        off += q;
        s0off[r] = off;
        off += s;
        s1off[r] = off;
        off += s;
        if (!tw_off.count(d.n)) {
            tw_off[d.n] = off;
            off += up((size_t)d.n * 16);
        }
    }
    // task lists, run-major
    b.xoff0.assign(nruns, 0);
    b.zoff0.assign(nruns, 0);
    for (int r = 0; r < nruns; ++r) {
        BRun &R = b.host[r];
        b.xoff0[r] = (int)b.xfull.size();
        for (long k = 0; k < x_tasks(R.n); ++k) b.xfull.push_back(BTask{r, (int)k});
        b.zoff0[r] = (int)b.yfull.size();
        for (long k = 0; k < yz_tasks(R.n, R.W, R.ntx); ++k) b.yfull.push_back(BTask{r, (int)k});
        R.xoff = b.xoff0[r];
        R.nxt = (int)x_tasks(R.n);
        R.zoff = b.zoff0[r];
        R.nzt = (int)yz_tasks(R.n, R.W, R.ntx);
    }
    const size_t o_runs = off;
    off += up(sizeof(BRun) * nruns);
    const size_t o_xt = off;
    off += up(sizeof(BTask) * b.xfull.size());
    const size_t o_yt = off;
    off += up(sizeof(BTask) * b.yfull.size());
    const size_t o_cnt = off;
    off += up(2 * sizeof(int));
    const size_t o_pa = off;
    off += up(2 * sizeof(double) * b.xfull.size());
    const size_t o_pc = off;
    off += up(2 * sizeof(double) * b.yfull.size());
    hipError_t e = hipMalloc(&b.arena, off);
    if (e != hipSuccess) return bfail(KG_E_NOMEM, "batch arena of " + std::to_string(off) + " bytes");
    char *base = (char *)b.arena;
    for (int r = 0; r < nruns; ++r) {
        b.host[r].Q = base + qoff[r];
        b.host[r].S0 = base + s0off[r];
        b.host[r].S1 = base + s1off[r];
        b.host[r].tw = base + tw_off[b.host[r].n];
    }
    b.d_runs = (BRun *)(base + o_runs);
    b.d_xt = (BTask *)(base + o_xt);
    b.d_yt = (BTask *)(base + o_yt);
    b.d_cnt = (int *)(base + o_cnt);
    b.d_pa = (double *)(base + o_pa);
    b.d_pc = (double *)(base + o_pc);
    for (auto &kv : tw_off) {
        const int n = kv.first;
        std::vector<double> tw(2 * (size_t)n);
        for (int j = 0; j < n; ++j) {
            const double ang = 2.0 * M_PI * (double)j / (double)n;
            tw[2 * j] = std::cos(ang);
            tw[2 * j + 1] = -std::sin(ang);
        }
        BCHK(hipMemcpyAsync(base + kv.second, tw.data(), tw.size() * sizeof(double),
                            hipMemcpyHostToDevice, b.st));
        BCHK(hipStreamSynchronize(b.st));
    }
    const int cnt[2] = {(int)b.xfull.size(), (int)b.yfull.size()};
    BCHK(hipMemcpyAsync(b.d_runs, b.host.data(), sizeof(BRun) * nruns, hipMemcpyHostToDevice, b.st));
    BCHK(hipMemcpyAsync(b.d_xt, b.xfull.data(), sizeof(BTask) * b.xfull.size(), hipMemcpyHostToDevice, b.st));
    BCHK(hipMemcpyAsync(b.d_yt, b.yfull.data(), sizeof(BTask) * b.yfull.size(), hipMemcpyHostToDevice, b.st));
    BCHK(hipMemcpyAsync(b.d_cnt, cnt, sizeof cnt, hipMemcpyHostToDevice, b.st));
    BCHK(hipStreamSynchronize(b.st));
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b.grid = 2 * cus;  // two 56 KB-LDS workgroups fit a CU
    return KG_OK;
}

void launch_x(Batch &b, hipStream_t st, int mode, int want, int cube)
{
    dim3 g(b.grid), t(256);
    switch (mode) {
    case X_STEP: hipLaunchKernelGGL((kb_xpass<double, X_STEP>), g, t, 0, st, b.d_runs, b.xl(), b.d_pa, want, cube); break;
    case X_REDUCE: hipLaunchKernelGGL((kb_xpass<double, X_REDUCE>), g, t, 0, st, b.d_runs, b.xl(), b.d_pa, want, cube); break;
    case X_GAUSS: hipLaunchKernelGGL((kb_xpass<double, X_GAUSS>), g, t, 0, st, b.d_runs, b.xl(), b.d_pa, want, cube); break;
    }
}
void launch_y(Batch &b, hipStream_t st, int dir, int want)
{
    dim3 g(b.grid), t(256);
    if (dir < 0)
        hipLaunchKernelGGL((kb_ypass<double, -1>), g, t, 0, st, b.d_runs, b.yl(), want);
    else
        hipLaunchKernelGGL((kb_ypass<double, 1>), g, t, 0, st, b.d_runs, b.yl(), want);
}
void launch_z(Batch &b, hipStream_t st, int mode, int want, int sel)
{
    dim3 g(b.grid), t(256);
    switch (mode) {
    case Z_STEP: hipLaunchKernelGGL((kb_zpass<double, Z_STEP>), g, t, 0, st, b.d_runs, b.yl(), b.d_pc, want, sel, 0); break;
    case Z_FWD_STATE: hipLaunchKernelGGL((kb_zpass<double, Z_FWD_STATE>), g, t, 0, st, b.d_runs, b.yl(), b.d_pc, want, sel, 0); break;
    case Z_START: hipLaunchKernelGGL((kb_zpass<double, Z_START>), g, t, 0, st, b.d_runs, b.yl(), b.d_pc, want, sel, 0); break;
    case Z_INV_STATE: hipLaunchKernelGGL((kb_zpass<double, Z_INV_STATE>), g, t, 0, st, b.d_runs, b.yl(), b.d_pc, want, sel, 0); break;
    case Z_PAIR: hipLaunchKernelGGL((kb_zpass<double, Z_PAIR>), g, t, 0, st, b.d_runs, b.yl(), b.d_pc, want, sel, 0); break;
    }
}
void launch_fin(Batch &b, hipStream_t st, int mode, int want)
{
    const int g = std::min(b.nruns, 2048);
    hipLaunchKernelGGL(kb_finalize, dim3(g), dim3(256), 0, st, b.d_runs, b.nruns, b.d_pa, b.d_pc, mode, want);
}

// Initial levels, energy of the initial pair and the first working field.
kg_status init(Batch &b)
{
    hipStream_t st = b.st;
    launch_x(b, st, X_GAUSS, 0, 1);  // N^0 = F[u0^3] -> S1
    launch_y(b, st, -1, 0);
    launch_z(b, st, Z_FWD_STATE, 0, 1);
    launch_x(b, st, X_GAUSS, 0, 0);  // v^0 = F[u0] -> S0
    launch_y(b, st, -1, 0);
    launch_z(b, st, Z_FWD_STATE, 0, 2);
    launch_z(b, st, Z_START, 0, 5);  // v^{-1} (u_t = 0) -> S1
    launch_z(b, st, Z_PAIR, 0, 5);   // linear energy of (v^{-1}, v^0)
    launch_z(b, st, Z_INV_STATE, 0, 3);  // Q4 of u^{-1}
    launch_y(b, st, 1, 0);
    launch_x(b, st, X_REDUCE, 0, 0);
    launch_fin(b, st, BF_INIT, 0);
    launch_z(b, st, Z_INV_STATE, 0, 4);  // working field of v^0
    launch_y(b, st, 1, 0);
    BCHK(hipGetLastError());
    return KG_OK;
}

void enqueue_steps(Batch &b, hipStream_t st, int nsteps)
{
    for (int i = 0; i < nsteps; ++i) {
        launch_x(b, st, X_STEP, 0, 0);
        launch_y(b, st, -1, 0);
        launch_z(b, st, Z_STEP, 0, 0);
        launch_y(b, st, 1, 0);
        launch_fin(b, st, BF_STEP, 0);
    }
}

kg_status make_graph(Batch &b, int G)
{
    BCHK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    enqueue_steps(b, b.cap, G);
    BCHK(hipStreamEndCapture(b.cap, &g));
    hipError_t e = hipGraphInstantiate(&b.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b.gexec = nullptr;
        return bfail(KG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return KG_OK;
}

// Rebuild the task lists for the runs whose flag equals `want` (the run
// table on the device must be idle).  Returns the number of such runs.
kg_status compact(Batch &b, int want, int &nsel)
{
    BCHK(hipMemcpyAsync(b.host.data(), b.d_runs, sizeof(BRun) * b.nruns, hipMemcpyDeviceToHost, b.st));
    BCHK(hipStreamSynchronize(b.st));
    std::vector<BTask> xt, yt;
    nsel = 0;
    for (int r = 0; r < b.nruns; ++r) {
        BRun &R = b.host[r];
        if (R.flag != want) continue;
        ++nsel;
        const int nx = R.nxt, nz = R.nzt;
        R.xoff = (int)xt.size();
        xt.insert(xt.end(), b.xfull.begin() + b.xoff0[r], b.xfull.begin() + b.xoff0[r] + nx);
        R.zoff = (int)yt.size();
        yt.insert(yt.end(), b.yfull.begin() + b.zoff0[r], b.yfull.begin() + b.zoff0[r] + nz);
    }
    const int cnt[2] = {(int)xt.size(), (int)yt.size()};
    if (!xt.empty())
        BCHK(hipMemcpyAsync(b.d_xt, xt.data(), sizeof(BTask) * xt.size(), hipMemcpyHostToDevice, b.st));
    if (!yt.empty())
        BCHK(hipMemcpyAsync(b.d_yt, yt.data(), sizeof(BTask) * yt.size(), hipMemcpyHostToDevice, b.st));
    BCHK(hipMemcpyAsync(b.d_cnt, cnt, sizeof cnt, hipMemcpyHostToDevice, b.st));
    BCHK(hipMemcpyAsync(b.d_runs, b.host.data(), sizeof(BRun) * b.nruns, hipMemcpyHostToDevice, b.st));
    BCHK(hipStreamSynchronize(b.st));
    return KG_OK;
}

// Whole sweep of one batch; per-run tile widths W.
kg_status run_batch(const kg_run_desc *runs, int nruns, const std::vector<int> &W, double L, int G,
                    hipStream_t st, std::vector<BRun> &result, double *seconds)
{
    Batch b;
    b.st = st;
    kg_status s = setup(b, runs, nruns, W, L);
    if (s != KG_OK) return s;
    if ((s = init(b)) != KG_OK) return s;
    BCHK(hipStreamSynchronize(st));
    if ((s = make_graph(b, G)) != KG_OK) return s;
    int max_steps = 0;
    for (int r = 0; r < nruns; ++r) max_steps = std::max(max_steps, runs[r].max_steps);
    const auto t0 = std::chrono::steady_clock::now();
    int active = 0, tasks_live = (int)b.yfull.size();
    if ((s = compact(b, 0, active)) != KG_OK) return s;
    long done = 0;
    while (active > 0 && done < max_steps) {
        const int left = max_steps - (int)done;
        if (left >= G) {
            BCHK(hipGraphLaunch(b.gexec, st));
            done += G;
        } else {
            enqueue_steps(b, st, left);
            BCHK(hipGetLastError());
            done += left;
        }
        // drop retired runs from the task lists once enough of them are gone
        BCHK(hipMemcpyAsync(b.host.data(), b.d_runs, sizeof(BRun) * nruns, hipMemcpyDeviceToHost, st));
        BCHK(hipStreamSynchronize(st));
        int live_tasks = 0, a = 0;
        for (int r = 0; r < nruns; ++r)
            if (b.host[r].flag == 0) {
                ++a;
                live_tasks += b.host[r].nzt;
            }
        active = a;
        if (active > 0 && live_tasks < 0.8 * tasks_live) {
            if ((s = compact(b, 0, active)) != KG_OK) return s;
            tasks_live = live_tasks;
        }
    }
    BCHK(hipStreamSynchronize(st));
    const auto t1 = std::chrono::steady_clock::now();
    if (seconds) *seconds = std::chrono::duration<double>(t1 - t0).count();
    // Q4 of the last level of finished runs, for E_final
    int fin = 0;
    if ((s = compact(b, 2, fin)) != KG_OK) return s;
    if (fin > 0) {
        launch_x(b, st, X_REDUCE, 2, 0);
        launch_fin(b, st, BF_FINAL, 2);
        BCHK(hipGetLastError());
    }
    BCHK(hipMemcpyAsync(b.host.data(), b.d_runs, sizeof(BRun) * nruns, hipMemcpyDeviceToHost, st));
    BCHK(hipStreamSynchronize(st));
    result = b.host;
    return KG_OK;
}

// Tile width per size: measured on a small batch of stable runs of that size.
int tune_width(int n, double L, hipStream_t st, double dt)
{
    const int R = 16, steps = 20;
    std::vector<kg_run_desc> d(R);
    for (int i = 0; i < R; ++i) d[i] = kg_run_desc{n, 0.5, 1.0, 1.1, 0.9, dt, steps, 0.0};
    int best = 8;
    double tbest = 1e30;
    for (int w : {4, 8}) {
        std::vector<int> W(R, w);
        std::vector<BRun> res;
        double secs = 0;
        if (run_batch(d.data(), R, W, L, 10, st, res, &secs) != KG_OK) continue;
        if (secs < tbest) {
            tbest = secs;
            best = w;
        }
    }
    return best;
}

}  // namespace

extern "C" {

const char *kg_batch_last_error(void) { return g_err.c_str(); }

kg_status kg_batch_run(const kg_run_desc *runs, int nruns, kg_run_result *out,
                       const kg_batch_opts *opts, void *hip_stream)
{
    g_err.clear();
    if (!runs || !out || nruns <= 0) return bfail(KG_E_INVALID, "no runs");
    for (int r = 0; r < nruns; ++r) {
        const kg_run_desc &d = runs[r];
        if (!batch_size_ok(d.n)) return bfail(KG_E_UNSUPPORTED_SIZE, "run " + std::to_string(r));
        if (!(d.dt > 0) || !std::isfinite(d.dt) || d.max_steps < 0 || !std::isfinite(d.A) ||
            !(d.sx > 0) || !(d.sy > 0) || !(d.sz > 0))
            return bfail(KG_E_INVALID, "run " + std::to_string(r));
    }
    const double L = opts && opts->L > 0 ? opts->L : 8.0 * M_PI;
    const int G = opts && opts->graph_steps > 0 ? opts->graph_steps : 10;
    hipStream_t st = (hipStream_t)hip_stream;

    // tile width per size: cache, autotuner, default 8
    std::string cpath;
    if (opts && opts->tune_cache) cpath = opts->tune_cache;
    else if (const char *e = std::getenv("KG_TUNE_CACHE")) cpath = e;
    auto cache = load_cache(cpath);
    std::map<int, int> width;
    bool changed = false;
    for (int r = 0; r < nruns; ++r) {
        const int n = runs[r].n;
        if (width.count(n)) continue;
        auto it = cache.find(cache_key(n));
        if (it != cache.end() && (it->second == 4 || it->second == 8)) {
            width[n] = it->second;
        } else if (opts && opts->tune) {
            width[n] = tune_width(n, L, st, runs[r].dt);
            cache[cache_key(n)] = width[n];
            changed = true;
        } else {
            width[n] = 8;
        }
    }
    if (changed) save_cache(cpath, cache);
    std::vector<int> W(nruns);
    for (int r = 0; r < nruns; ++r) W[r] = width[runs[r].n];

    std::vector<BRun> res;
    kg_status s = run_batch(runs, nruns, W, L, G, st, res, opts ? opts->seconds : nullptr);
    if (s != KG_OK) return s;
    for (int r = 0; r < nruns; ++r) {
        const BRun &R = res[r];
        kg_run_result &o = out[r];
        o.blew_up = R.flag == 1;
        o.steps_done = R.flag == 1 ? R.blow_step : R.max_steps;
        o.t_blowup = R.flag == 1 ? R.blow_step * R.dt : -1.0;
        o.E0 = R.E0;
        o.E_final = R.flag == 1 ? std::nan("") : R.E_final;
        o.max_abs_u = R.maxu_max;
        if (R.max_steps == 0) {
            o.E0 = std::nan("");
            o.E_final = std::nan("");
        }
    }
    return KG_OK;
}

}  // extern "C"
