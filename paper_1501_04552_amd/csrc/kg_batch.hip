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

std::string cache_key(int n, const char *what) { return "fp64/" + std::to_string(n) + "/" + what; }

// Launch parameters of one grid size: tile width of the y and z passes,
// persistent workgroups per CU (at most what the LDS allows), and fields
// per chunk of the size class in MB (0: the whole class).  A graph replays
// all its steps on one chunk before the next, the size classes running as
// concurrent branches.  Defaults: on MI355X, for the {48,64,96,128}^3 sweep,
// 400 MB chunks measured 17% faster than whole classes (50-200 MB lose to
// per-launch overheads, 800 MB and more to cache misses).  The autotuner
// replaces them per size; KG_BATCH_CHUNK_MB overrides the chunk size.
struct Tune {
    int W = 8;
    int wpc = 4;
    double chunk_mb = 400;
};

double chunk_bytes(const Tune &t)
{
    if (const char *e = std::getenv("KG_BATCH_CHUNK_MB")) return std::atof(e) * 1e6;
    return t.chunk_mb * 1e6;
}

// ---------------------------------------------------------------------------
// One batch: runs grouped in size classes, one persistent kernel per class
// ---------------------------------------------------------------------------

// The tasks one set of launches covers: a whole size class, or a chunk of
// it (consecutive runs of the class's task lists).
struct View {
    BList xl, yl;       // x-pass and y/z-pass tasks (count in device memory)
    double *pa, *pc;    // partial slots of the lists' first tasks
    double *fa, *fc;    // the class's partial arrays (the finalize indexes them)
    const int *list;    // run indices for the finalize
    int nlist;
    int gx, gyz;        // persistent grid sizes
};

// Launchers of one (grid size, tile width).
struct Launch {
    void (*x)(const View &, hipStream_t, BRun *, int mode, int want, int cube);
    void (*y)(const View &, hipStream_t, BRun *, int dir, int want);
    void (*z)(const View &, hipStream_t, BRun *, int mode, int want, int sel);
    long (*x_tasks)();
    long (*yz_tasks)(int ntx);
    int x_lds, yz_lds;
};

struct Class {
    int n = 0, W = 0;
    Tune tune;
    const Launch *L = nullptr;
    std::vector<int> runs;            // run indices
    std::vector<BTask> xfull, yfull;  // full task lists (run-major)
    std::vector<int> xoff0, zoff0;    // offsets of each run's tasks (by position in `runs`)
    BTask *d_xt = nullptr, *d_yt = nullptr;
    int *d_cnt = nullptr, *d_list = nullptr;
    double *d_pa = nullptr, *d_pc = nullptr;
    int gx = 0, gyz = 0;  // persistent grid sizes
    int nlist = 0;        // runs in d_list
    int *d_ccnt = nullptr;     // task counts of the chunks (x, y/z per chunk)
    std::vector<View> chunks;  // the class in chunks of consecutive runs
    hipStream_t side = nullptr;
    hipEvent_t ev = nullptr;
    View whole() const
    {
        return View{BList{d_xt, d_cnt}, BList{d_yt, d_cnt + 1}, d_pa, d_pc, d_pa, d_pc, d_list, nlist,
                    gx, gyz};
    }
};

template <int N, int W>
struct LaunchImpl {
    static void x(const View &c, hipStream_t st, BRun *runs, int mode, int want, int cube)
    {
        dim3 g(c.gx), t(256);
        switch (mode) {
        case X_STEP: hipLaunchKernelGGL((kb_xpass<double, N, X_STEP>), g, t, 0, st, runs, c.xl, c.pa, want, cube); break;
        case X_REDUCE: hipLaunchKernelGGL((kb_xpass<double, N, X_REDUCE>), g, t, 0, st, runs, c.xl, c.pa, want, cube); break;
        case X_GAUSS: hipLaunchKernelGGL((kb_xpass<double, N, X_GAUSS>), g, t, 0, st, runs, c.xl, c.pa, want, cube); break;
        }
    }
    static void y(const View &c, hipStream_t st, BRun *runs, int dir, int want)
    {
        dim3 g(c.gyz), t(256);
        if (dir < 0)
            hipLaunchKernelGGL((kb_ypass<double, N, W, -1>), g, t, 0, st, runs, c.yl, want);
        else
            hipLaunchKernelGGL((kb_ypass<double, N, W, 1>), g, t, 0, st, runs, c.yl, want);
    }
    static void z(const View &c, hipStream_t st, BRun *runs, int mode, int want, int sel)
    {
        dim3 g(c.gyz), t(256);
        switch (mode) {
        case Z_STEP: hipLaunchKernelGGL((kb_zpass<double, N, W, Z_STEP>), g, t, 0, st, runs, c.yl, c.pc, want, sel); break;
        case Z_FWD_STATE: hipLaunchKernelGGL((kb_zpass<double, N, W, Z_FWD_STATE>), g, t, 0, st, runs, c.yl, c.pc, want, sel); break;
        case Z_START: hipLaunchKernelGGL((kb_zpass<double, N, W, Z_START>), g, t, 0, st, runs, c.yl, c.pc, want, sel); break;
        case Z_INV_STATE: hipLaunchKernelGGL((kb_zpass<double, N, W, Z_INV_STATE>), g, t, 0, st, runs, c.yl, c.pc, want, sel); break;
        case Z_PAIR: hipLaunchKernelGGL((kb_zpass<double, N, W, Z_PAIR>), g, t, 0, st, runs, c.yl, c.pc, want, sel); break;
        }
    }
    static long xt() { return XCfg<double, N>::blocks(); }
    static long yzt(int ntx) { return (long)ntx * ((N + YZCfg<N, W>::B - 1) / YZCfg<N, W>::B); }
    static constexpr Launch tab = {x, y, z, xt, yzt,
                                   XCfg<double, N>::PPB * XCfg<double, N>::RS * 16,
                                   W * YZCfg<N, W>::B * lslots<N>() * 16};
};

const Launch *launch_table(int n, int W)
{
    switch (n * 16 + W) {
#define KG_TCASE(NN)                                              \
    case NN * 16 + 4: return &LaunchImpl<NN, 4>::tab;             \
    case NN * 16 + 8: return &LaunchImpl<NN, 8>::tab;
        KG_TCASE(32)
        KG_TCASE(48)
        KG_TCASE(64)
        KG_TCASE(96)
        KG_TCASE(128)
#undef KG_TCASE
    }
    return nullptr;
}

struct Batch {
    hipStream_t st = nullptr;
    int nruns = 0;
    std::vector<BRun> host;  // run table (host copy)
    std::vector<size_t> bytes;  // fields of each run (Q and both levels)
    int cus = 256, lds_cu = 160 * 1024;
    // persistent grids: wpc 256-thread workgroups per CU, no more than the
    // LDS lets a CU hold (reductions add ~2 KB), no more than the tasks
    int grid(int lds, long tasks, int wpc) const
    {
        const int per_cu = std::max(1, std::min(wpc, lds_cu / (lds + 2048)));
        return (int)std::max(1L, std::min((long)per_cu * cus, tasks));
    }
    std::vector<Class> cls;
    void *arena = nullptr;
    BRun *d_runs = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    hipGraphExec_t gexec = nullptr;
    int *d_active = nullptr;        // active runs after the last replay (device)
    int *h_active = nullptr;        // ... copied by each replay into pinned host memory
    hipEvent_t done_ev[2] = {nullptr, nullptr};  // replays in flight
    ~Batch()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        for (hipEvent_t e : done_ev)
            if (e) (void)hipEventDestroy(e);
        if (h_active) (void)hipHostFree(h_active);
        for (Class &c : cls) {
            if (c.side) (void)hipStreamDestroy(c.side);
            if (c.ev) (void)hipEventDestroy(c.ev);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (cap) (void)hipStreamDestroy(cap);
        if (arena) (void)hipFree(arena);
    }
};

kg_status setup(Batch &b, const kg_run_desc *runs, int nruns, const std::map<int, Tune> &tune,
                double L)
{
    b.nruns = nruns;
    b.host.assign(nruns, BRun{});
    std::map<int, size_t> tw_off;  // one twiddle table per size
    std::map<std::pair<int, int>, int> cls_of;
    size_t off = 0;
    std::vector<size_t> qoff(nruns), s0off(nruns), s1off(nruns);
    for (int r = 0; r < nruns; ++r) {
        BRun &R = b.host[r];
        const kg_run_desc &d = runs[r];
        R.n = d.n;
        R.H = d.n / 2 + 1;
        R.W = tune.at(d.n).W;
        R.ntx = (R.H + R.W - 1) / R.W;
        R.P = ((R.ntx * R.W + 7) / 8) * 8;
        R.flag = 0;  // runs of zero steps retire after the set-up (run_batch)
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
        b.bytes.push_back(q + 2 * s);
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
        auto key = std::make_pair(R.n, R.W);
        if (!cls_of.count(key)) {
            cls_of[key] = (int)b.cls.size();
            b.cls.emplace_back();
            b.cls.back().n = R.n;
            b.cls.back().W = R.W;
            b.cls.back().L = launch_table(R.n, R.W);
            b.cls.back().tune = tune.at(d.n);
        }
        b.cls[cls_of[key]].runs.push_back(r);
    }
    // per class: task lists (run-major), partial offsets relative to the class
    std::vector<size_t> o_xt(b.cls.size()), o_yt(b.cls.size()), o_cnt(b.cls.size()),
        o_list(b.cls.size()), o_pa(b.cls.size()), o_pc(b.cls.size()), o_ccnt(b.cls.size());
    for (size_t k = 0; k < b.cls.size(); ++k) {
        Class &c = b.cls[k];
        for (size_t q = 0; q < c.runs.size(); ++q) {
            BRun &R = b.host[c.runs[q]];
            c.xoff0.push_back((int)c.xfull.size());
            for (long t = 0; t < c.L->x_tasks(); ++t) c.xfull.push_back(BTask{c.runs[q], (int)t});
            c.zoff0.push_back((int)c.yfull.size());
            for (long t = 0; t < c.L->yz_tasks(R.ntx); ++t) c.yfull.push_back(BTask{c.runs[q], (int)t});
            R.xoff = c.xoff0.back();
            R.nxt = (int)c.L->x_tasks();
            R.zoff = c.zoff0.back();
            R.nzt = (int)c.L->yz_tasks(R.ntx);
        }
        o_xt[k] = off;
        off += up(sizeof(BTask) * c.xfull.size());
        o_yt[k] = off;
        off += up(sizeof(BTask) * c.yfull.size());
        o_cnt[k] = off;
        off += up(2 * sizeof(int));
        o_list[k] = off;
        off += up(sizeof(int) * c.runs.size());
        o_pa[k] = off;
        off += up(2 * sizeof(double) * c.xfull.size());
        o_pc[k] = off;
        off += up(2 * sizeof(double) * c.yfull.size());
        o_ccnt[k] = off;
        off += up(2 * sizeof(int) * c.runs.size());
    }
    const size_t o_runs = off;
    off += up(sizeof(BRun) * nruns);
    const size_t o_active = off;
    off += up(sizeof(int));
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
    b.d_active = (int *)(base + o_active);
    BCHK(hipHostMalloc((void **)&b.h_active, sizeof(int), hipHostMallocDefault));
    *b.h_active = nruns;
    for (hipEvent_t &e : b.done_ev) BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&b.lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    for (size_t k = 0; k < b.cls.size(); ++k) {
        Class &c = b.cls[k];
        c.d_xt = (BTask *)(base + o_xt[k]);
        c.d_yt = (BTask *)(base + o_yt[k]);
        c.d_cnt = (int *)(base + o_cnt[k]);
        c.d_list = (int *)(base + o_list[k]);
        c.d_pa = (double *)(base + o_pa[k]);
        c.d_pc = (double *)(base + o_pc[k]);
        c.d_ccnt = (int *)(base + o_ccnt[k]);
        c.nlist = (int)c.runs.size();
        c.gx = b.grid(c.L->x_lds, (long)c.xfull.size(), c.tune.wpc);
        c.gyz = b.grid(c.L->yz_lds, (long)c.yfull.size(), c.tune.wpc);
        const int cnt[2] = {(int)c.xfull.size(), (int)c.yfull.size()};
        BCHK(hipMemcpyAsync(c.d_xt, c.xfull.data(), sizeof(BTask) * c.xfull.size(), hipMemcpyHostToDevice, b.st));
        BCHK(hipMemcpyAsync(c.d_yt, c.yfull.data(), sizeof(BTask) * c.yfull.size(), hipMemcpyHostToDevice, b.st));
        BCHK(hipMemcpyAsync(c.d_cnt, cnt, sizeof cnt, hipMemcpyHostToDevice, b.st));
        BCHK(hipMemcpyAsync(c.d_list, c.runs.data(), sizeof(int) * c.runs.size(), hipMemcpyHostToDevice, b.st));
        BCHK(hipStreamSynchronize(b.st));
    }
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
    BCHK(hipMemcpyAsync(b.d_runs, b.host.data(), sizeof(BRun) * nruns, hipMemcpyHostToDevice, b.st));
    BCHK(hipStreamSynchronize(b.st));
    return KG_OK;
}

void launch_fin(Batch &b, const View &v, hipStream_t st, int mode, int want)
{
    const int g = std::max(1, std::min(v.nlist, 1024));
    hipLaunchKernelGGL(kb_finalize, dim3(g), dim3(256), 0, st, b.d_runs, v.list, v.nlist, v.fa, v.fc,
                       mode, want);
}

// Initial levels, energy of the initial pair and the first working field.
kg_status init(Batch &b)
{
    hipStream_t st = b.st;
    for (const Class &cl : b.cls) {
        const Launch &L = *cl.L;
        const View c = cl.whole();
        L.x(c, st, b.d_runs, X_GAUSS, 0, 1);  // N^0 = F[u0^3] -> S1
        L.y(c, st, b.d_runs, -1, 0);
        L.z(c, st, b.d_runs, Z_FWD_STATE, 0, 1);
        L.x(c, st, b.d_runs, X_GAUSS, 0, 0);  // v^0 = F[u0] -> S0
        L.y(c, st, b.d_runs, -1, 0);
        L.z(c, st, b.d_runs, Z_FWD_STATE, 0, 2);
        L.z(c, st, b.d_runs, Z_START, 0, 5);  // v^{-1} (u_t = 0) -> S1
        L.z(c, st, b.d_runs, Z_PAIR, 0, 5);   // linear energy of (v^{-1}, v^0)
        L.z(c, st, b.d_runs, Z_INV_STATE, 0, 3);  // Q4 of u^{-1}
        L.y(c, st, b.d_runs, 1, 0);
        L.x(c, st, b.d_runs, X_REDUCE, 0, 0);
        launch_fin(b, c, st, BF_INIT, 0);
        L.z(c, st, b.d_runs, Z_INV_STATE, 0, 4);  // working field of v^0
        L.y(c, st, b.d_runs, 1, 0);
    }
    BCHK(hipGetLastError());
    return KG_OK;
}

// nsteps steps of a class, chunk by chunk: a chunk's fields stay in the
// memory-side cache across its steps (runs are independent, so the order of
// steps across chunks is free).
void enqueue_steps(Batch &b, const Class &cl, hipStream_t st, int nsteps)
{
    const Launch &L = *cl.L;
    for (const View &c : cl.chunks) {
        for (int i = 0; i < nsteps; ++i) {
            L.x(c, st, b.d_runs, X_STEP, 0, 0);
            L.y(c, st, b.d_runs, -1, 0);
            L.z(c, st, b.d_runs, Z_STEP, 0, 0);
            L.y(c, st, b.d_runs, 1, 0);
            launch_fin(b, c, st, BF_STEP, 0);
        }
    }
}

// G steps of every size class as concurrent branches of one graph.
kg_status make_graph(Batch &b, int G)
{
    BCHK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    BCHK(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
    for (Class &c : b.cls) {
        BCHK(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
    }
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    BCHK(hipEventRecord(b.fork, b.cap));
    for (Class &c : b.cls) {
        BCHK(hipStreamWaitEvent(c.side, b.fork, 0));
        enqueue_steps(b, c, c.side, G);
        BCHK(hipEventRecord(c.ev, c.side));
        BCHK(hipStreamWaitEvent(b.cap, c.ev, 0));
    }
    // the replay ends by counting the active runs into pinned host memory
    hipLaunchKernelGGL(kb_count_active, dim3(1), dim3(256), 0, b.cap, b.d_runs, b.nruns, b.d_active);
    BCHK(hipMemcpyAsync(b.h_active, b.d_active, sizeof(int), hipMemcpyDeviceToHost, b.cap));
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
    nsel = 0;
    for (Class &c : b.cls) {
        std::vector<BTask> xt, yt;
        std::vector<int> list;
        for (size_t q = 0; q < c.runs.size(); ++q) {
            BRun &R = b.host[c.runs[q]];
            if (R.flag != want) continue;
            list.push_back(c.runs[q]);
            R.xoff = (int)xt.size();
            xt.insert(xt.end(), c.xfull.begin() + c.xoff0[q], c.xfull.begin() + c.xoff0[q] + R.nxt);
            R.zoff = (int)yt.size();
            yt.insert(yt.end(), c.yfull.begin() + c.zoff0[q], c.yfull.begin() + c.zoff0[q] + R.nzt);
        }
        nsel += (int)list.size();
        // the finalize grid reads nlist; the full list stays allocated
        c.nlist = (int)list.size();
        c.gx = b.grid(c.L->x_lds, (long)xt.size(), c.tune.wpc);
        c.gyz = b.grid(c.L->yz_lds, (long)yt.size(), c.tune.wpc);
        // chunks of consecutive runs of about chunk_bytes() of fields each
        std::vector<int> ccnt;
        c.chunks.clear();
        const double cap = chunk_bytes(c.tune);
        for (size_t a = 0; a < list.size();) {
            size_t e = a + 1;
            double acc = (double)b.bytes[list[a]];
            while (e < list.size() && cap > 0 && acc + b.bytes[list[e]] <= cap) acc += b.bytes[list[e++]];
            if (cap <= 0) e = list.size();
            const BRun &A = b.host[list[a]], &Z = b.host[list[e - 1]];
            const int xa = A.xoff, xb = Z.xoff + Z.nxt, ya = A.zoff, yb = Z.zoff + Z.nzt;
            const int k = (int)c.chunks.size();
            ccnt.push_back(xb - xa);
            ccnt.push_back(yb - ya);
            c.chunks.push_back(View{BList{c.d_xt + xa, c.d_ccnt + 2 * k}, BList{c.d_yt + ya, c.d_ccnt + 2 * k + 1},
                                    c.d_pa + 2 * xa, c.d_pc + 2 * ya, c.d_pa, c.d_pc, c.d_list + a,
                                    (int)(e - a), b.grid(c.L->x_lds, xb - xa, c.tune.wpc),
                                    b.grid(c.L->yz_lds, yb - ya, c.tune.wpc)});
            a = e;
        }
        if (!ccnt.empty())
            BCHK(hipMemcpyAsync(c.d_ccnt, ccnt.data(), sizeof(int) * ccnt.size(), hipMemcpyHostToDevice, b.st));
        const int cnt[2] = {(int)xt.size(), (int)yt.size()};
        if (!xt.empty())
            BCHK(hipMemcpyAsync(c.d_xt, xt.data(), sizeof(BTask) * xt.size(), hipMemcpyHostToDevice, b.st));
        if (!yt.empty())
            BCHK(hipMemcpyAsync(c.d_yt, yt.data(), sizeof(BTask) * yt.size(), hipMemcpyHostToDevice, b.st));
        if (!list.empty())
            BCHK(hipMemcpyAsync(c.d_list, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, b.st));
        BCHK(hipMemcpyAsync(c.d_cnt, cnt, sizeof cnt, hipMemcpyHostToDevice, b.st));
    }
    BCHK(hipMemcpyAsync(b.d_runs, b.host.data(), sizeof(BRun) * b.nruns, hipMemcpyHostToDevice, b.st));
    BCHK(hipStreamSynchronize(b.st));
    return KG_OK;
}

// Whole sweep of one batch with per-size launch parameters.
kg_status run_batch(const kg_run_desc *runs, int nruns, const std::map<int, Tune> &tune, double L,
                    int G, hipStream_t st, std::vector<BRun> &result, double *seconds)
{
    Batch b;
    b.st = st;
    kg_status s = setup(b, runs, nruns, tune, L);
    if (s != KG_OK) return s;
    if ((s = init(b)) != KG_OK) return s;
    BCHK(hipStreamSynchronize(st));
    // Runs of zero steps are set up like the others, so the final reduction
    // finds their level 0 (its energy, max|u| and blow-up test), and retire
    // before the first step.
    bool unstepped = false;
    for (int r = 0; r < nruns; ++r) unstepped = unstepped || runs[r].max_steps == 0;
    if (unstepped) {
        BCHK(hipMemcpyAsync(b.host.data(), b.d_runs, sizeof(BRun) * nruns, hipMemcpyDeviceToHost, st));
        BCHK(hipStreamSynchronize(st));
        for (BRun &R : b.host)
            if (R.flag == 0 && R.max_steps == 0) R.flag = 2;
        BCHK(hipMemcpyAsync(b.d_runs, b.host.data(), sizeof(BRun) * nruns, hipMemcpyHostToDevice, st));
        BCHK(hipStreamSynchronize(st));
    }
    int max_steps = 0;
    for (int r = 0; r < nruns; ++r) max_steps = std::max(max_steps, runs[r].max_steps);
    const auto t0 = std::chrono::steady_clock::now();
    int active = 0;
    if ((s = compact(b, 0, active)) != KG_OK) return s;
    // the graph reads the finalize grids' run counts at capture: capture after
    // the first compaction, and recapture whenever a compaction changes them
    if ((s = make_graph(b, G)) != KG_OK) return s;
    long tasks_live = 0;
    for (const Class &c : b.cls) tasks_live += (long)c.nlist;
    long done = 0;
    // Replays stay queued one ahead: after launching replay k the host waits
    // for replay k-1 and reads the active count it (or a later replay) left
    // in pinned memory, so the GPU never idles on the host.  A replay that
    // runs after every run has retired does nothing (retired runs' tasks are
    // skipped on the device).
    long k = 0;
    while (active > 0 && done < max_steps) {
        const int left = max_steps - (int)done;
        if (left >= G) {
            BCHK(hipGraphLaunch(b.gexec, st));
            BCHK(hipEventRecord(b.done_ev[k & 1], st));
            done += G;
            if (k > 0) {
                BCHK(hipEventSynchronize(b.done_ev[(k - 1) & 1]));
                active = *(volatile int *)b.h_active;
            }
            ++k;
        } else {
            for (const Class &c : b.cls) enqueue_steps(b, c, st, left);
            BCHK(hipGetLastError());
            done += left;
            BCHK(hipStreamSynchronize(st));
            k = 0;
        }
        // drop retired runs from the task lists once enough of them are gone
        if (active > 0 && active < 0.8 * tasks_live && done < max_steps) {
            BCHK(hipStreamSynchronize(st));
            k = 0;
            if ((s = compact(b, 0, active)) != KG_OK) return s;
            tasks_live = active;
            (void)hipGraphExecDestroy(b.gexec);
            b.gexec = nullptr;
            for (Class &c : b.cls) {
                (void)hipStreamDestroy(c.side);
                (void)hipEventDestroy(c.ev);
                c.side = nullptr;
                c.ev = nullptr;
            }
            (void)hipEventDestroy(b.fork);
            (void)hipStreamDestroy(b.cap);
            b.fork = nullptr;
            b.cap = nullptr;
            if ((s = make_graph(b, G)) != KG_OK) return s;
        }
    }
    BCHK(hipStreamSynchronize(st));
    const auto t1 = std::chrono::steady_clock::now();
    if (seconds) *seconds = std::chrono::duration<double>(t1 - t0).count();
    // Q4 of the last level of finished runs, for E_final
    int fin = 0;
    if ((s = compact(b, 2, fin)) != KG_OK) return s;
    if (fin > 0) {
        for (const Class &c : b.cls) {
            if (c.nlist == 0) continue;
            c.L->x(c.whole(), st, b.d_runs, X_REDUCE, 2, 0);
            launch_fin(b, c.whole(), st, BF_FINAL, 2);
        }
        BCHK(hipGetLastError());
    }
    BCHK(hipMemcpyAsync(b.host.data(), b.d_runs, sizeof(BRun) * nruns, hipMemcpyDeviceToHost, st));
    BCHK(hipStreamSynchronize(st));
    result = b.host;
    return KG_OK;
}

// Launch parameters for the sizes in `todo`, measured on the batch itself:
// the sizes share the GPU as concurrent graph branches, so a size's best
// parameters depend on the others'.  A trial steps a sample of the batch's
// runs (every k-th, at most 128, at most 60 steps each), twice, and counts
// its faster time; coordinate descent over the sizes (largest first) and,
// per size, tile width, workgroups per CU and chunk size keeps a new setting
// only when it beats the best so far by 2% (run-to-run noise of a trial is
// about that large, and the defaults are the best single setting measured
// for the whole sweep).
std::map<int, Tune> tune_mix(const kg_run_desc *runs, int nruns, std::map<int, Tune> tune,
                             const std::vector<int> &todo, double L, hipStream_t st)
{
    const int step = std::max(1, nruns / 128);
    std::vector<kg_run_desc> d;
    for (int r = 0; r < nruns && (int)d.size() < 128; r += step) {
        d.push_back(runs[r]);
        d.back().max_steps = std::min(d.back().max_steps, 60);
    }
    double tbest = 1e30;
    auto trial = [&](const std::map<int, Tune> &m) {
        double best = 1e30;
        for (int rep = 0; rep < 2; ++rep) {
            std::vector<BRun> res;
            double secs = 0;
            if (run_batch(d.data(), (int)d.size(), m, L, 10, st, res, &secs) != KG_OK) return false;
            best = std::min(best, secs);
        }
        if (best < 0.98 * tbest || tbest == 1e30) {
            tbest = best;
            return true;
        }
        return false;
    };
    trial(tune);
    std::vector<int> order = todo;
    std::sort(order.begin(), order.end(), [](int a, int b) { return a > b; });
    for (int n : order) {
        auto attempt = [&](Tune t) {
            std::map<int, Tune> m = tune;
            m[n] = t;
            if (trial(m)) tune = m;
        };
        for (int w : {4, 8})
            if (w != tune[n].W) attempt(Tune{w, tune[n].wpc, tune[n].chunk_mb});
        for (int wpc : {2, 3, 4})
            if (wpc != tune[n].wpc) attempt(Tune{tune[n].W, wpc, tune[n].chunk_mb});
        for (double mb : {200.0, 400.0, 800.0})
            if (mb != tune[n].chunk_mb) attempt(Tune{tune[n].W, tune[n].wpc, mb});
    }
    return tune;
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

    // launch parameters per size: cache, autotuner, defaults
    std::string cpath;
    if (opts && opts->tune_cache) cpath = opts->tune_cache;
    else if (const char *e = std::getenv("KG_TUNE_CACHE")) cpath = e;
    auto cache = load_cache(cpath);
    std::map<int, Tune> tune;
    std::vector<int> todo;  // sizes without cached parameters
    for (int r = 0; r < nruns; ++r) {
        const int n = runs[r].n;
        if (tune.count(n)) continue;
        auto w = cache.find(cache_key(n, "W")), p = cache.find(cache_key(n, "wpc")),
             c = cache.find(cache_key(n, "chunk_mb"));
        tune[n] = Tune{};
        if (w != cache.end() && p != cache.end() && c != cache.end() &&
            (w->second == 4 || w->second == 8) && p->second >= 1 && p->second <= 4 &&
            c->second >= 0) {
            tune[n].W = w->second;
            tune[n].wpc = p->second;
            tune[n].chunk_mb = c->second;
        } else {
            todo.push_back(n);
        }
    }
    if (opts && opts->tune && !todo.empty()) {
        tune = tune_mix(runs, nruns, tune, todo, L, st);
        for (int n : todo) {
            cache[cache_key(n, "W")] = tune[n].W;
            cache[cache_key(n, "wpc")] = tune[n].wpc;
            cache[cache_key(n, "chunk_mb")] = (int)tune[n].chunk_mb;
        }
        save_cache(cpath, cache);
    }

    std::vector<BRun> res;
    kg_status s = run_batch(runs, nruns, tune, L, G, st, res, opts ? opts->seconds : nullptr);
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
    }
    return KG_OK;
}

}  // extern "C"
