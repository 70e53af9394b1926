// kg_api.hip -- C-ABI of the Klein-Gordon spectral stepper (declared in kg.h).
//
// Host-side plan logic: workspace carving, the initialisation sequence, the
// step loop (four passes and a finalize per step of eq. (2), Sec. 1.1.2),
// the energy of Sec. 1.1, checkpointing and the test/measurement hooks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "kg_plan.hpp"

using namespace kg;

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Tile width of the y and z passes: W complex columns give 16*W-byte (FP64)
// or 8*W-byte (FP32) row segments per wavefront access.  Whole 128-byte
// lines stream at 5.5 TB/s where 64-byte segments reach 4.5 (measured at
// 512^3 FP64).  KG_TILE_W overrides the default for experiments.
int tile_width(int precision)
{
    const int def = precision == KG_FP32 ? 16 : 8;
    const char *e = std::getenv("KG_TILE_W");
    if (e) {
        const int w = std::atoi(e);
        if ((precision == KG_FP64 && (w == 4 || w == 8)) || (precision == KG_FP32 && (w == 8 || w == 16)))
            return w;
    }
    return def;
}

// Padding, in bytes, between consecutive z planes of the working field, a
// multiple of 128 so rows stay line-aligned; KG_PLANE_PAD overrides.  The z
// pass reads and writes one 128-byte segment per plane along each column;
// unpadded plane pitches are multiples of 64 KiB at the large grids (512^3:
// 33 * 64 KiB real, 4 MiB complex), which crowds those accesses onto the
// same memory channels.  256 bytes measured best at 512^3 (z pass FP64 real
// 1.10 -> 1.02 ms, complex 2.32 -> 1.98 ms); any pad from 128 to 768 bytes
// helps, while 1 KiB and 4 KiB pads do not.
long plane_pad_bytes()
{
    const char *e = std::getenv("KG_PLANE_PAD");
    if (e) {
        const long b = std::atol(e);
        if (b >= 0 && b % 128 == 0 && b <= (1L << 20)) return b;
    }
    return 256;
}

std::unique_ptr<Ops> make_ops(int n, int precision, int W)
{
    if (precision == KG_FP64) return make_ops_f64(n, W);
    if (precision == KG_FP32) return make_ops_f32(n, W);
    return nullptr;
}

// Grid sizes: powers of two 8..512 and three times a power of two 24..384.
bool size_ok(int n)
{
    const int b = (n % 3 == 0) ? n / 3 : n;
    const bool pow2 = b > 0 && (b & (b - 1)) == 0;
    return pow2 && ((n % 3 != 0 && n >= 8 && n <= 512) || (n % 3 == 0 && n >= 24 && n <= 384));
}

struct Layout {
    int n, H, W, ntx, P;
    long PZ;
    size_t esz, q, s, tw, pa, pc, sub, rec, ctl, total;
    long nA, nC;
};

bool layout(const kg_params *p, Layout &lo)
{
    if (!p || !size_ok(p->n) || (p->precision != KG_FP64 && p->precision != KG_FP32)) return false;
    lo.n = p->n;
    lo.H = p->complex_field ? p->n : p->n / 2 + 1;  // full spectrum of a complex field
    lo.W = tile_width(p->precision);
    lo.ntx = (lo.H + lo.W - 1) / lo.W;
    lo.esz = p->precision == KG_FP32 ? 8 : 16;
    // kx rows padded to whole 128-byte lines and to whole tiles
    const int per_line = (int)(128 / lo.esz);
    lo.P = ((lo.ntx * lo.W + per_line - 1) / per_line) * per_line;
    lo.PZ = (long)lo.n * lo.P + plane_pad_bytes() / (long)lo.esz;
    auto ops = make_ops(p->n, p->precision, lo.W);
    lo.nA = ops->x_blocks(p->complex_field ? 1 : 0);
    lo.nC = ops->z_blocks(lo.ntx);
    if (lo.nC < PAIR_BLOCKS) lo.nC = PAIR_BLOCKS;
    lo.q = up((size_t)lo.n * lo.PZ * lo.esz);
    lo.s = up((size_t)lo.n * lo.ntx * lo.n * lo.W * lo.esz);
    lo.tw = up((size_t)lo.n * lo.esz);
    lo.pa = up((size_t)lo.nA * 2 * sizeof(double));
    lo.pc = up((size_t)lo.nC * 2 * sizeof(double));
    lo.sub = up((size_t)RSUB * 3 * sizeof(double));
    lo.rec = up((size_t)RING * sizeof(Rec));
    lo.ctl = up(sizeof(Ctl));
    lo.total = lo.q + 2 * lo.s + lo.tw + lo.pa + lo.pc + lo.sub + lo.rec + lo.ctl;
    return true;
}

// Planes per slab of the y-inverse / x / y-forward chain of a step.  A field
// larger than the GPU's 256 MB memory-side cache is processed in slabs of
// about SLAB_BYTES, so that each slab stays cached from the y-inverse through
// the x pass to the y-forward pass; smaller fields are one slab.  Captured
// steps run alternate slabs on two streams, so two slabs share the cache: at
// 512^3 on MI355X 120 MB slabs measured best (one stream: 240 MB, 2% slower).
// KG_SLAB_MB overrides the slab size (0: one slab).
constexpr double SLAB_BYTES = 120e6;
constexpr double CACHE_BYTES = 256e6;

int slab_planes(const Layout &lo, const Ops &ops)
{
    const double plane = (double)lo.PZ * lo.esz;
    double target = (double)lo.n * plane > CACHE_BYTES ? SLAB_BYTES : 0.0;
    if (const char *e = std::getenv("KG_SLAB_MB")) target = std::atof(e) * 1e6;
    const int q = ops.slab_quantum();
    if (!(target > 0) || target >= lo.n * plane) return lo.n;
    int nz = (int)(target / plane) / q * q;
    if (nz < q) nz = q;
    // even slabs: as many as the target size asks for, as equal as q allows
    const int nslab = (lo.n + nz - 1) / nz;
    nz = ((lo.n + nslab - 1) / nslab + q - 1) / q * q;
    return nz < lo.n ? nz : lo.n;
}

kg_status fail(kg_plan_s *pl, kg_status s, const char *msg)
{
    if (pl) pl->err = msg;
    return s;
}

kg_status hip_fail(kg_plan_s *pl, hipError_t e, const char *where)
{
    if (pl) pl->err = std::string(where) + ": " + hipGetErrorString(e);
    return KG_E_HIP;
}

#define HIPCHK(pl, expr)                                           \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail((pl), e_, #expr);    \
    } while (0)

#define LAUNCHCHK(pl)                                              \
    do {                                                           \
        hipError_t e_ = hipGetLastError();                         \
        if (e_ != hipSuccess) return hip_fail((pl), e_, "launch"); \
    } while (0)

Plan &P(kg_plan_s *p) { return *p; }

// Doubles per field: n^3, or 2 n^3 interleaved (re, im) for a complex field.
size_t field_doubles(const kg_plan_s *pl) { return (size_t)pl->n * pl->n * pl->n * (pl->cf ? 2 : 1); }

// Device copy of a field given on the host or the device.
struct DevField {
    double *d = nullptr;
    bool own = false;
    ~DevField()
    {
        if (own && d) (void)hipFree(d);
    }
};

kg_status to_device(kg_plan_s *pl, const double *src, int on_device, DevField &f)
{
    if (!src) return KG_OK;
    if (on_device) {
        f.d = const_cast<double *>(src);
        return KG_OK;
    }
    const size_t bytes = field_doubles(pl) * sizeof(double);
    HIPCHK(pl, hipMalloc((void **)&f.d, bytes));
    f.own = true;
    HIPCHK(pl, hipMemcpyAsync(f.d, src, bytes, hipMemcpyHostToDevice, pl->stream));
    return KG_OK;
}

// Half spectrum (host or device) -> Q, and back.
kg_status spec_in(kg_plan_s *pl, const double *spec, int on_device)
{
    const size_t bytes = (size_t)pl->n * pl->n * pl->H * 16;
    double *d = const_cast<double *>(spec);
    if (!on_device) {
        HIPCHK(pl, hipMalloc((void **)&d, bytes));
        HIPCHK(pl, hipMemcpyAsync(d, spec, bytes, hipMemcpyHostToDevice, pl->stream));
    }
    pl->ops->spec_to_q(*pl, d);
    LAUNCHCHK(pl);
    if (!on_device) {
        HIPCHK(pl, hipStreamSynchronize(pl->stream));
        HIPCHK(pl, hipFree(d));
    }
    return KG_OK;
}

kg_status spec_out(kg_plan_s *pl, double *spec, int on_device)
{
    const size_t bytes = (size_t)pl->n * pl->n * pl->H * 16;
    double *d = spec;
    if (!on_device) HIPCHK(pl, hipMalloc((void **)&d, bytes));
    pl->ops->q_to_spec(*pl, d);
    LAUNCHCHK(pl);
    if (!on_device) {
        HIPCHK(pl, hipMemcpyAsync(spec, d, bytes, hipMemcpyDeviceToHost, pl->stream));
        HIPCHK(pl, hipStreamSynchronize(pl->stream));
        HIPCHK(pl, hipFree(d));
    }
    return KG_OK;
}

// What stopped a run: a blow-up, or the energy alarm (kg_set_energy_alarm).
kg_status stop_status(const Ctl &c) { return c.flag == 2 ? KG_E_ENERGY : KG_BLOWUP; }

kg_status read_ctl(kg_plan_s *pl, Ctl &c)
{
    HIPCHK(pl, hipMemcpyAsync(&c, pl->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(pl, hipStreamSynchronize(pl->stream));
    return KG_OK;
}

// Two-launch fixed-order reduction of the partials into a record (see k_finalize).
void finalize(Plan &p, int nC, double thr, int mode)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(RSUB), dim3(256), 0, p.stream, p.partA, (int)p.nA,
                       p.partC, nC, p.sub, p.ctl, mode != 2 ? 1 : 0);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RSUB), 0, p.stream, p.sub, p.rec, p.ctl, thr,
                       p.escale, p.h3, p.chi, mode);
}

// Q <- inverse z transform of level S (scaled by 1/M): the resting state of
// the working field between steps, which the next step's y-inverse pass
// starts from.  It equals what the z pass of a step leaves for the level it
// stores (same values, same transform), so it also restores Q after calls
// that use Q as scratch.
kg_status prepare_q(kg_plan_s *pl, const void *S, const void *Ssub = nullptr)
{
    Plan &p = P(pl);
    p.ops->z(p, Z_INV_STATE, nullptr, const_cast<void *>(S), p.invM, 0, Ssub);
    LAUNCHCHK(pl);
    return KG_OK;
}

// Q (resting state of level S) <- the level's half spectrum inverse
// transformed along z and y: what an x pass turns into u.
kg_status physical_q(kg_plan_s *pl, const void *S, const void *Ssub = nullptr)
{
    kg_status s = prepare_q(pl, S, Ssub);
    if (s != KG_OK) return s;
    Plan &p = P(pl);
    p.ops->y(p, 1, false);
    LAUNCHCHK(pl);
    return KG_OK;
}

bool increment(const Plan &p) { return p.p.precision == KG_FP32; }

// State buffers the step from level m reads and writes: (v^m, v^{m-1})
// alternate between S[0] and S[1] for FP64; FP32 keeps (v, Delta) in place.
void step_levels(Plan &p, long m, void *&Sc, void *&Sp)
{
    if (increment(p)) {
        Sc = p.S[0];
        Sp = p.S[1];
    } else {
        Sc = p.S[m & 1];
        Sp = p.S[(m + 1) & 1];
    }
}

// The stored level v^{n-back} (back = 0 or 1) after the control block `c`,
// as a buffer S minus an optional Ssub.  After a blow-up at level n the FP32
// buffers hold v^{n+1} and Delta^{n+1}, so v^n = v - Delta.
void stored_level(Plan &p, const Ctl &c, int back, const void *&S, const void *&Ssub)
{
    Ssub = nullptr;
    if (increment(p)) {
        S = p.S[0];
        if (c.flag || back == 1) Ssub = p.S[1];
    } else {
        S = p.S[(c.step - back) & 1];
    }
}

// Statistics of the newest level n = c.step (Q4^n, max|u^n|) into rec[n]:
// the y-inverse of the resting field, an x pass with reductions only, then
// the resting field rebuilt from the stored level.  The step from level n
// overwrites rec[n] with the same values plus its energy.
kg_status newest_level_stats(kg_plan_s *pl, const Ctl &c)
{
    Plan &p = P(pl);
    p.ops->y(p, 1, false);
    p.ops->x(p, X_REDUCE, nullptr, nullptr, 0.0);
    finalize(p, 0, 0.0, 1);
    const void *S, *Ssub;
    stored_level(p, c, 0, S, Ssub);
    kg_status s = prepare_q(pl, S, Ssub);
    if (s != KG_OK) return s;
    HIPCHK(pl, hipStreamSynchronize(p.stream));
    return KG_OK;
}

// E^{m-1/2} for levels m = first .. first+count-1 (energy of Sec. 1.1 of the
// pair (v^{m-1}, v^m)):  elin of the pair minus chi (Q4^{m-1} + Q4^m)/8.  The
// pair energies and Q4 come from the per-step records; the initial pair's
// from the control block; Q4 of the newest level is reduced on demand.
kg_status energies(kg_plan_s *pl, const Ctl &c, int first, int count, double *E)
{
    Plan &p = P(pl);
    if (count == 0) return KG_OK;
    const int last = first + count - 1;  // newest level asked for
    const int top = c.step;              // newest level (the blown one after a blow-up)
    if (last > top) return fail(pl, KG_E_INVALID, "energy of a level not reached");
    if (top - first + 1 > RING - 1) return fail(pl, KG_E_INVALID, "records not retained");
    if (last == top && !c.flag) {
        kg_status s = newest_level_stats(pl, c);
        if (s != KG_OK) return s;
    }
    std::vector<Rec> r(count + 1);
    for (int m = (first > 0 ? first - 1 : 0); m <= last; ++m)
        HIPCHK(pl, hipMemcpy(&r[m - first + 1], p.rec + (m & (RING - 1)), sizeof(Rec),
                             hipMemcpyDeviceToHost));
    for (int m = first; m <= last; ++m) {
        const Rec &cur = r[m - first + 1];
        const double elin = m == 0 ? c.elin_m : r[m - first].elin;
        const double q4p = m == 0 ? c.q4_m : r[m - first].q4;
        E[m - first] = elin - p.chi * (q4p + cur.q4) / 8.0;
    }
    return KG_OK;
}

kg_status prepare_graphs(Plan &p);  // defined with the step graphs below

// One forward 3D r2c transform of a real field into Q (x, then y; the z
// transform is done by the caller's z-pass mode).
void forward_xy(Plan &p, const double *d_real, bool cube, const double *d_minus = nullptr)
{
    p.ops->x(p, X_R2C, d_real, nullptr, cube ? 1.0 : 0.0, d_minus);
    p.ops->y(p, -1, false);
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------

extern "C" {

const char *kg_status_str(kg_status s)
{
    switch (s) {
    case KG_OK: return "KG_OK";
    case KG_E_INVALID: return "KG_E_INVALID";
    case KG_E_UNSUPPORTED_SIZE: return "KG_E_UNSUPPORTED_SIZE";
    case KG_E_NOMEM: return "KG_E_NOMEM";
    case KG_E_HIP: return "KG_E_HIP";
    case KG_BLOWUP: return "KG_BLOWUP";
    case KG_E_ENERGY: return "KG_E_ENERGY";
    }
    return "unknown status";
}

const char *kg_last_error(const kg_plan_t *plan) { return plan ? plan->err.c_str() : "no plan"; }

size_t kg_workspace_bytes(const kg_params *p)
{
    Layout lo;
    if (!p || !(p->dt > 0)) return 0;
    return layout(p, lo) ? lo.total : 0;
}

kg_status kg_plan(const kg_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream,
                  kg_plan_t **out)
{
    if (!p || !out) return KG_E_INVALID;
    *out = nullptr;
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return KG_E_INVALID;
    if (p->precision != KG_FP64 && p->precision != KG_FP32) return KG_E_INVALID;
    if (!size_ok(p->n)) return KG_E_UNSUPPORTED_SIZE;
    Layout lo;
    if (!layout(p, lo)) return KG_E_INVALID;
    if (d_workspace && ws_bytes < lo.total) return KG_E_NOMEM;

    kg_plan_s *pl = new (std::nothrow) kg_plan_s();
    if (!pl) return KG_E_NOMEM;
    pl->p = *p;
    pl->n = lo.n;
    pl->cf = p->complex_field ? 1 : 0;
    pl->dkc = p->dealias ? p->n / 3 : 0;
    pl->H = lo.H;
    pl->W = lo.W;
    pl->ntx = lo.ntx;
    pl->P = lo.P;
    pl->PZ = lo.PZ;
    pl->esz = lo.esz;
    pl->ops = make_ops(p->n, p->precision, lo.W);
    if (!pl->ops) {
        delete pl;
        return KG_E_UNSUPPORTED_SIZE;
    }
    pl->zslab = slab_planes(lo, *pl->ops);
    pl->L = p->L > 0 ? p->L : 8.0 * M_PI;
    const double h = pl->L / pl->n;
    pl->h3 = h * h * h;
    const double ks = 2.0 * M_PI / pl->L;
    pl->ks2 = ks * ks;
    const double M = (double)pl->n * pl->n * pl->n;
    pl->invM = 1.0 / M;
    pl->escale = pl->h3 / (2.0 * M);
    pl->chi = p->linear_only ? 0.0 : 1.0;
    pl->stream = (hipStream_t)hip_stream;
    pl->nA = lo.nA;
    pl->nC = lo.nC;
    pl->q_bytes = lo.q;
    pl->s_bytes = lo.s;

    if (d_workspace) {
        pl->ws = d_workspace;
        pl->ws_bytes = ws_bytes;
    } else {
        hipError_t e = hipMalloc(&pl->ws, lo.total);
        if (e != hipSuccess) {
            delete pl;
            return KG_E_NOMEM;
        }
        pl->own_ws = true;
        pl->ws_bytes = lo.total;
    }
    char *c = (char *)pl->ws;
    pl->Q = c;
    c += lo.q;
    pl->S[0] = c;
    c += lo.s;
    pl->S[1] = c;
    c += lo.s;
    pl->tw = c;
    c += lo.tw;
    pl->partA = (double *)c;
    c += lo.pa;
    pl->partC = (double *)c;
    c += lo.pc;
    pl->sub = (double *)c;
    c += lo.sub;
    pl->rec = (Rec *)c;
    c += lo.rec;
    pl->ctl = (Ctl *)c;

    // Twiddle table exp(-2 pi i j / n), each entry from cos/sin in double
    // (rounded once to float for the FP32 path).
    std::vector<double> tw(2 * (size_t)pl->n);
    std::vector<float> twf(2 * (size_t)pl->n);
    for (int j = 0; j < pl->n; ++j) {
        const double ang = 2.0 * M_PI * (double)j / (double)pl->n;
        tw[2 * j] = std::cos(ang);
        tw[2 * j + 1] = -std::sin(ang);
        twf[2 * j] = (float)tw[2 * j];
        twf[2 * j + 1] = (float)tw[2 * j + 1];
    }
    Ctl c0{};
    c0.blow_step = -1;
    const bool f32 = p->precision == KG_FP32;
    hipError_t e = hipMemcpyAsync(pl->tw, f32 ? (const void *)twf.data() : (const void *)tw.data(),
                                  tw.size() * (f32 ? sizeof(float) : sizeof(double)),
                                  hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) {
        kg_destroy(pl);
        return KG_E_HIP;
    }
    *out = pl;
    return KG_OK;
}

void kg_destroy(kg_plan_t *plan)
{
    if (!plan) return;
    for (hipEvent_t e : plan->tev) (void)hipEventDestroy(e);
    for (hipGraphExec_t g : plan->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipGraphExec_t g : plan->gexec1)
        if (g) (void)hipGraphExecDestroy(g);
    if (plan->cap) (void)hipStreamDestroy(plan->cap);
    if (plan->cap2) (void)hipStreamDestroy(plan->cap2);
    if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
    if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
    if (plan->own_ws && plan->ws) (void)hipFree(plan->ws);
    delete plan;
}

kg_status kg_set_state(kg_plan_t *plan, const double *u0, const double *aux, int mode,
                       int on_device)
{
    if (!plan || !u0) return KG_E_INVALID;
    if (mode != KG_INIT_VELOCITY && mode != KG_INIT_TWO_LEVEL)
        return fail(plan, KG_E_INVALID, "unknown init mode");
    if (mode == KG_INIT_TWO_LEVEL && !aux)
        return fail(plan, KG_E_INVALID, "two-level start needs u^{-1}");
    Plan &p = P(plan);
    kg_status s;
    DevField du0, daux;
    if ((s = to_device(plan, u0, on_device, du0)) != KG_OK) return s;
    if ((s = to_device(plan, aux, on_device, daux)) != KG_OK) return s;

    Ctl c0{};
    c0.blow_step = -1;
    c0.e_tol = p.e_tol;
    HIPCHK(plan, hipMemcpyAsync(p.ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice, p.stream));
    // FP64: v^m lives in S[m % 2] (v^0 -> S[0], v^{-1} -> S[1]).
    // FP32: S[0] = v^0, S[1] = Delta^0 = v^0 - v^{-1}.
    void *S0 = p.S[0], *S1 = p.S[1];
    if (mode == KG_INIT_VELOCITY) {
        if (p.chi != 0.0) {  // N^0 = F[u0^3] -> S1
            forward_xy(p, du0.d, true);
            p.ops->z(p, Z_FWD_STATE, S1, nullptr, 1.0, 0);
        }
        forward_xy(p, du0.d, false);  // v^0 -> S0
        p.ops->z(p, Z_FWD_STATE, S0, nullptr, 1.0, 0);
        if (daux.d) forward_xy(p, daux.d, false);  // F_xy[u_t0] in Q
        p.ops->z(p, Z_START, S1, S0, 1.0, daux.d ? 1 : 0);
    } else {
        forward_xy(p, du0.d, false);
        p.ops->z(p, Z_FWD_STATE, S0, nullptr, 1.0, 0);
        if (increment(p))
            forward_xy(p, du0.d, false, daux.d);  // F[u^0 - u^{-1}]
        else
            forward_xy(p, daux.d, false);
        p.ops->z(p, Z_FWD_STATE, S1, nullptr, 1.0, 0);
    }
    LAUNCHCHK(plan);
    // Energy of the initial pair: linear part of (v^{-1}, v^0) and Q4 of u^{-1}.
    if (increment(p)) {
        p.ops->pair_energy(p, S0, S1);
        if ((s = physical_q(plan, S0, S1)) != KG_OK) return s;
    } else {
        p.ops->pair_energy(p, S1, S0);
        if ((s = physical_q(plan, S1)) != KG_OK) return s;
    }
    p.ops->x(p, X_REDUCE, nullptr, nullptr, 0.0);
    finalize(p, PAIR_BLOCKS, 0.0, 2);
    LAUNCHCHK(plan);
    if ((s = prepare_q(plan, S0)) != KG_OK) return s;
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    if ((s = prepare_graphs(p)) != KG_OK) return s;
    p.steps = 0;
    p.ready = true;
    return KG_OK;
}

}  // extern "C"

namespace {

// Kernel kinds of a step, in the order of kg_kernel_times.
enum { K_X = 0, K_YF = 1, K_Z = 2, K_YI = 3, K_FIN = 4 };

// Enqueue the kernels of step m (levels v^{m-1}, v^m -> v^{m+1}) on stream st:
// per slab of z planes the inverse y pass (from the resting state), the x
// pass and the forward y pass; then the z pass (which leaves the next
// resting state) and the finalize.  `mark(kind)` runs after each launch
// (timing).  With a `side` stream the odd slabs' chains run on it, forked
// from and joined back to st: slabs are independent, so one slab's kernels
// fill the tail of another's (the results are the same).
template <typename F>
void enqueue_step(Plan &p, long m, hipStream_t st, F &&mark, hipStream_t side = nullptr)
{
    void *Sc, *Sp;
    step_levels(p, m, Sc, Sp);
    hipStream_t keep = p.stream;
    const bool two = side && p.zslab < p.n;
    if (two) {
        (void)hipEventRecord(p.ev_fork, st);
        (void)hipStreamWaitEvent(side, p.ev_fork, 0);
    }
    int slab = 0;
    for (int z0 = 0; z0 < p.n; z0 += p.zslab, ++slab) {
        const int nz = p.n - z0 < p.zslab ? p.n - z0 : p.zslab;
        p.stream = two && (slab & 1) ? side : st;
        p.ops->y(p, 1, true, z0, nz);
        mark(K_YI);
        p.ops->x(p, X_STEP, nullptr, nullptr, p.chi, nullptr, z0, nz);
        mark(K_X);
        p.ops->y(p, -1, true, z0, nz);
        mark(K_YF);
    }
    p.stream = st;
    if (two) {
        (void)hipEventRecord(p.ev_join, side);
        (void)hipStreamWaitEvent(st, p.ev_join, 0);
    }
    p.ops->z(p, Z_STEP, Sp, Sc, p.invM, 0);
    mark(K_Z);
    finalize(p, (int)p.ops->z_step_parts(p.ntx), p.p.blowup_threshold, 0);
    mark(K_FIN);
    p.stream = keep;
}

constexpr int GRAPH_STEPS = 8;  // steps per captured graph (even: parity returns)

// Streams the slab chain of a captured step runs on (KG_SLAB_STREAMS, 1 or 2).
int slab_streams()
{
    if (const char *e = std::getenv("KG_SLAB_STREAMS")) return std::atoi(e) > 1 ? 2 : 1;
    return 2;
}

// The second capture stream of a step's slab chain (created on first use),
// or null when the chain is one slab or KG_SLAB_STREAMS asks for one stream.
hipStream_t slab_side(Plan &p)
{
    if (slab_streams() < 2 || p.zslab >= p.n) return nullptr;
    if (!p.cap2 && hipStreamCreateWithFlags(&p.cap2, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (!p.ev_fork && hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    if (!p.ev_join && hipEventCreateWithFlags(&p.ev_join, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    return p.cap2;
}

// The graph of `len` steps (GRAPH_STEPS or 1) starting at a level of parity
// `par`, captured once on the plan's private stream, uploaded, and replayed
// on the plan's stream.
kg_status step_graph(Plan &p, int par, int len, hipGraphExec_t &out)
{
    hipGraphExec_t &ge = len == GRAPH_STEPS ? p.gexec[par] : p.gexec1[par];
    if (!ge) {
        if (!p.cap) HIPCHK(&p, hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking));
        hipStream_t side = slab_side(p);
        hipGraph_t g = nullptr;
        HIPCHK(&p, hipStreamBeginCapture(p.cap, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < len; ++i) enqueue_step(p, par + i, p.cap, [](int) {}, side);
        hipError_t e = hipStreamEndCapture(p.cap, &g);
        if (e != hipSuccess) return hip_fail(&p, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ge = nullptr;
            return hip_fail(&p, e, "hipGraphInstantiate");
        }
        // move the graph to the device now, not at its first launch
        HIPCHK(&p, hipGraphUpload(ge, p.stream));
    }
    out = ge;
    return KG_OK;
}

// Capture every step graph a kg_step call can launch (both parities, whole
// and single steps), so that no later kg_step pays for capture.
kg_status prepare_graphs(Plan &p)
{
    hipGraphExec_t ge;
    for (int par = 0; par < 2; ++par)
        for (int len : {GRAPH_STEPS, 1}) {
            kg_status s = step_graph(p, par, len, ge);
            if (s != KG_OK) return s;
        }
    return KG_OK;
}

}  // namespace

extern "C" {

kg_status kg_step(kg_plan_t *plan, int nsteps, unsigned flags, int *steps_done)
{
    if (!plan || nsteps < 0) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    const bool timed = (flags & KG_STEP_TIMED) != 0;
    if (!timed) {
        // whole graphs of GRAPH_STEPS steps, then single-step graphs
        int done = 0;
        while (done < nsteps) {
            const int len = nsteps - done >= GRAPH_STEPS ? GRAPH_STEPS : 1;
            hipGraphExec_t ge;
            kg_status s = step_graph(p, (int)((p.steps + done) & 1), len, ge);
            if (s != KG_OK) return s;
            HIPCHK(plan, hipGraphLaunch(ge, p.stream));
            done += len;
        }
        p.steps += nsteps;
        if (flags & KG_STEP_SYNC) {
            Ctl c;
            kg_status s = read_ctl(plan, c);
            if (s != KG_OK) return s;
            if (steps_done) *steps_done = c.step;
            if (c.flag) return stop_status(c);
        }
        return KG_OK;
    }
    // KG_STEP_TIMED: an event after every launch; the time between an event
    // and the next is charged to the kind of the launch in between.
    const int nslab = (p.n + p.zslab - 1) / p.zslab;
    const size_t per_step = (size_t)3 * nslab + 3;  // launches + 1
    std::vector<int> kinds;
    const size_t need = per_step * nsteps;
    while (p.tev.size() < need) {
        hipEvent_t e;
        HIPCHK(plan, hipEventCreate(&e));
        p.tev.push_back(e);
    }
    kinds.reserve(need);
    hipError_t rec_err = hipSuccess;
    for (int i = 0; i < nsteps; ++i) {
        size_t k = per_step * i;
        rec_err = hipEventRecord(p.tev[k++], p.stream);
        enqueue_step(p, p.steps + i, p.stream, [&](int kind) {
            kinds.push_back(kind);
            if (rec_err == hipSuccess) rec_err = hipEventRecord(p.tev[k++], p.stream);
        });
        kinds.push_back(-1);  // no launch between this step's last event and the next step's first
        if (rec_err != hipSuccess) return hip_fail(plan, rec_err, "hipEventRecord");
    }
    LAUNCHCHK(plan);
    p.steps += nsteps;
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    for (int k = 0; k < 5; ++k) p.kt_ms[k] = 0.0;
    for (size_t e = 0; e + 1 < per_step * nsteps; ++e) {
        if (kinds[e] < 0) continue;
        float t = 0;
        HIPCHK(plan, hipEventElapsedTime(&t, p.tev[e], p.tev[e + 1]));
        p.kt_ms[kinds[e]] += t;
    }
    for (int k = 0; k < 5; ++k) p.kt_ms[k] = nsteps ? p.kt_ms[k] / nsteps : 0.0;
    p.kt_steps = nsteps;
    if (flags & KG_STEP_SYNC) {
        Ctl c;
        kg_status s = read_ctl(plan, c);
        if (s != KG_OK) return s;
        if (steps_done) *steps_done = c.step;
        if (c.flag) return stop_status(c);
    }
    return KG_OK;
}

kg_status kg_kernel_times(const kg_plan_t *plan, double ms[5], int *nsteps)
{
    if (!plan || !ms) return KG_E_INVALID;
    for (int k = 0; k < 5; ++k) ms[k] = plan->kt_ms[k];
    if (nsteps) *nsteps = plan->kt_steps;
    return KG_OK;
}

kg_status kg_energy(kg_plan_t *plan, double *E, double *t)
{
    if (!plan) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    if (c.flag) return stop_status(c);
    double e = 0.0;
    if ((s = energies(plan, c, c.step, 1, &e)) != KG_OK) return s;
    if (E) *E = e;
    if (t) *t = ((double)c.step - 0.5) * p.p.dt;
    return KG_OK;
}

kg_status kg_energies(kg_plan_t *plan, int first, int count, double *E)
{
    if (!plan || first < 0 || count < 0 || (count > 0 && !E)) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    return energies(plan, c, first, count, E);
}

kg_status kg_records(kg_plan_t *plan, int first, int count, double *elin, double *q4, double *maxu)
{
    if (!plan || first < 0 || count < 0) return KG_E_INVALID;
    Plan &p = P(plan);
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    const int done = c.flag ? c.step + 1 : c.step;  // a blown level has its record too
    if (first + count > done || done - first > RING)
        return fail(plan, KG_E_INVALID, "records not available");
    std::vector<Rec> all(RING);
    HIPCHK(plan, hipMemcpy(all.data(), p.rec, sizeof(Rec) * RING, hipMemcpyDeviceToHost));
    for (int i = 0; i < count; ++i) {
        const Rec &r = all[(first + i) & (RING - 1)];
        if (elin) elin[i] = r.elin;
        if (q4) q4[i] = r.q4;
        if (maxu) maxu[i] = r.maxu;
    }
    return KG_OK;
}

kg_status kg_stats(kg_plan_t *plan, int *steps_done, int *blown_up, int *blowup_step,
                   double *max_abs_u)
{
    if (!plan) return KG_E_INVALID;
    Plan &p = P(plan);
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    if (steps_done) *steps_done = c.step;
    if (blown_up) *blown_up = c.flag;
    if (blowup_step) *blowup_step = c.flag ? c.blow_step : -1;
    if (max_abs_u) {
        if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
        // the blown level's statistics were recorded by its step; otherwise
        // reduce the newest level now
        if (!c.flag && (s = newest_level_stats(plan, c)) != KG_OK) return s;
        Rec r;
        HIPCHK(plan, hipMemcpy(&r, p.rec + (c.step & (RING - 1)), sizeof r, hipMemcpyDeviceToHost));
        *max_abs_u = r.maxu;
    }
    return KG_OK;
}

kg_status kg_set_energy_alarm(kg_plan_t *plan, double rel_tol)
{
    if (!plan || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return KG_E_INVALID;
    Plan &p = P(plan);
    p.e_tol = rel_tol;
    // The step graphs read the tolerance from the control block as they run,
    // so no graph is captured again.
    HIPCHK(plan, hipMemcpyAsync((char *)p.ctl + offsetof(Ctl, e_tol), &p.e_tol, sizeof(double),
                                hipMemcpyHostToDevice, p.stream));
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    return KG_OK;
}

kg_status kg_get_u(kg_plan_t *plan, double *u_out, int on_device)
{
    if (!u_out) return KG_E_INVALID;
    return kg_get_state(plan, nullptr, u_out, on_device);
}

kg_status kg_get_state(kg_plan_t *plan, double *u_prev, double *u_cur, int on_device)
{
    if (!plan || (!u_prev && !u_cur)) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    if (c.flag && u_prev)
        return fail(plan, KG_E_INVALID, "after a blow-up the level before the blown one is overwritten");
    const size_t bytes = field_doubles(&p) * sizeof(double);
    double *outs[2] = {u_prev, u_cur};
    for (int which = 0; which < 2; ++which) {
        if (!outs[which]) continue;
        const void *S, *Ssub;
        stored_level(p, c, 1 - which, S, Ssub);
        if ((s = physical_q(plan, S, Ssub)) != KG_OK) return s;
        double *d = outs[which];
        if (!on_device) HIPCHK(plan, hipMalloc((void **)&d, bytes));
        p.ops->x(p, X_C2R, nullptr, d, 0.0);
        LAUNCHCHK(plan);
        if (!on_device) {
            HIPCHK(plan, hipMemcpyAsync(outs[which], d, bytes, hipMemcpyDeviceToHost, p.stream));
            HIPCHK(plan, hipStreamSynchronize(p.stream));
            HIPCHK(plan, hipFree(d));
        }
    }
    const void *S, *Ssub;
    stored_level(p, c, 0, S, Ssub);
    if ((s = prepare_q(plan, S, Ssub)) != KG_OK) return s;  // resting state again
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    return KG_OK;
}

kg_status kg_get_spectrum(kg_plan_t *plan, int which, double *out, int on_device)
{
    if (!plan || !out || (which != 0 && which != 1)) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    // The blown step's z pass has already written v^{n+1} over the level
    // before the blown one (FP64) or folded it into the increment (FP32).
    if (c.flag && which == 1)
        return fail(plan, KG_E_INVALID, "after a blow-up the level before the blown one is overwritten");
    const void *S, *Ssub;
    stored_level(p, c, which, S, Ssub);
    const size_t bytes = (size_t)p.n * p.n * p.H * 16;
    double *d = out;
    if (!on_device) HIPCHK(plan, hipMalloc((void **)&d, bytes));
    p.ops->state_to_spec(p, S, Ssub, d);
    LAUNCHCHK(plan);
    if (!on_device) {
        HIPCHK(plan, hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, p.stream));
        HIPCHK(plan, hipStreamSynchronize(p.stream));
        HIPCHK(plan, hipFree(d));
    } else {
        HIPCHK(plan, hipStreamSynchronize(p.stream));
    }
    return KG_OK;
}

// Saved state: header, both levels, control block and the newest record.
struct SaveHeader {
    uint64_t magic;
    int32_t n, precision, W, cf;
    double dt, L;
    int64_t s_bytes;
};
static const uint64_t KG_MAGIC = 0x4b47535441544532ull;  // "KGSTATE2"

size_t kg_state_bytes(const kg_plan_t *plan)
{
    if (!plan) return 0;
    return sizeof(SaveHeader) + 2 * plan->s_bytes + sizeof(Ctl) + sizeof(Rec);
}

kg_status kg_save_state(kg_plan_t *plan, void *host_buf, size_t bytes)
{
    if (!plan || !host_buf || bytes < kg_state_bytes(plan)) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    char *b = (char *)host_buf;
    SaveHeader h{KG_MAGIC, p.n, p.p.precision, p.W, p.cf, p.p.dt, p.L, (int64_t)p.s_bytes};
    std::memcpy(b, &h, sizeof h);
    b += sizeof h;
    HIPCHK(plan, hipMemcpy(b, p.S[0], p.s_bytes, hipMemcpyDeviceToHost));
    b += p.s_bytes;
    HIPCHK(plan, hipMemcpy(b, p.S[1], p.s_bytes, hipMemcpyDeviceToHost));
    b += p.s_bytes;
    std::memcpy(b, &c, sizeof c);
    b += sizeof c;
    Rec r{};
    if (c.step > 0)
        HIPCHK(plan, hipMemcpy(&r, p.rec + ((c.step - 1) & (RING - 1)), sizeof r, hipMemcpyDeviceToHost));
    std::memcpy(b, &r, sizeof r);
    return KG_OK;
}

kg_status kg_load_state(kg_plan_t *plan, const void *host_buf, size_t bytes)
{
    if (!plan || !host_buf || bytes < kg_state_bytes(plan)) return KG_E_INVALID;
    Plan &p = P(plan);
    const char *b = (const char *)host_buf;
    SaveHeader h;
    std::memcpy(&h, b, sizeof h);
    if (h.magic != KG_MAGIC || h.n != p.n || h.precision != p.p.precision || h.W != p.W ||
        h.cf != p.cf || h.s_bytes != (int64_t)p.s_bytes)
        return fail(plan, KG_E_INVALID, "saved state does not match this plan");
    b += sizeof h;
    HIPCHK(plan, hipMemcpy(p.S[0], b, p.s_bytes, hipMemcpyHostToDevice));
    b += p.s_bytes;
    HIPCHK(plan, hipMemcpy(p.S[1], b, p.s_bytes, hipMemcpyHostToDevice));
    b += p.s_bytes;
    Ctl c;
    std::memcpy(&c, b, sizeof c);
    b += sizeof c;
    c.e_tol = p.e_tol;  // the alarm setting belongs to the plan, not the saved run
    Rec r;
    std::memcpy(&r, b, sizeof r);
    HIPCHK(plan, hipMemcpy(p.ctl, &c, sizeof c, hipMemcpyHostToDevice));
    if (c.step > 0)
        HIPCHK(plan, hipMemcpy(p.rec + ((c.step - 1) & (RING - 1)), &r, sizeof r, hipMemcpyHostToDevice));
    const void *S, *Ssub;
    stored_level(p, c, 0, S, Ssub);
    kg_status s = prepare_q(plan, S, Ssub);
    if (s != KG_OK) return s;
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    if ((s = prepare_graphs(p)) != KG_OK) return s;
    p.steps = c.step;
    p.ready = true;
    return KG_OK;
}

// ---------------------------------------------------------------------------
// Test and measurement hooks
// ---------------------------------------------------------------------------

kg_status kg_debug_forward(kg_plan_t *plan, const double *u, double *spec, int on_device)
{
    if (!plan || !u || !spec) return KG_E_INVALID;
    Plan &p = P(plan);
    DevField du;
    kg_status s = to_device(plan, u, on_device, du);
    if (s != KG_OK) return s;
    p.ready = false;
    forward_xy(p, du.d, false);
    p.ops->z(p, Z_FWD_Q, nullptr, nullptr, 1.0, 0);
    LAUNCHCHK(plan);
    s = spec_out(plan, spec, on_device);
    if (s == KG_OK && on_device) HIPCHK(plan, hipStreamSynchronize(p.stream));
    return s;
}

kg_status kg_debug_inverse(kg_plan_t *plan, const double *spec, double *u, int on_device)
{
    if (!plan || !u || !spec) return KG_E_INVALID;
    Plan &p = P(plan);
    p.ready = false;
    kg_status s = spec_in(plan, spec, on_device);
    if (s != KG_OK) return s;
    p.ops->z(p, Z_INV_Q, nullptr, nullptr, 1.0, 0);
    p.ops->y(p, 1, false);
    const size_t bytes = field_doubles(&p) * sizeof(double);
    double *d = u;
    if (!on_device) HIPCHK(plan, hipMalloc((void **)&d, bytes));
    p.ops->x(p, X_C2R, nullptr, d, 0.0);
    LAUNCHCHK(plan);
    if (!on_device) {
        HIPCHK(plan, hipMemcpyAsync(u, d, bytes, hipMemcpyDeviceToHost, p.stream));
        HIPCHK(plan, hipStreamSynchronize(p.stream));
        HIPCHK(plan, hipFree(d));
    } else {
        HIPCHK(plan, hipStreamSynchronize(p.stream));
    }
    return KG_OK;
}

kg_status kg_debug_pass(kg_plan_t *plan, int pass, double *spec, int on_device)
{
    if (!plan || !spec || pass < 1 || pass > 4) return KG_E_INVALID;
    Plan &p = P(plan);
    p.ready = false;
    kg_status s = spec_in(plan, spec, on_device);
    if (s != KG_OK) return s;
    switch (pass) {
    case 1: p.ops->y(p, -1, false); break;
    case 2: p.ops->y(p, 1, false); break;
    case 3: p.ops->z(p, Z_FWD_Q, nullptr, nullptr, 1.0, 0); break;
    case 4: p.ops->z(p, Z_INV_Q, nullptr, nullptr, 1.0, 0); break;
    }
    LAUNCHCHK(plan);
    s = spec_out(plan, spec, on_device);
    if (s == KG_OK && on_device) HIPCHK(plan, hipStreamSynchronize(p.stream));
    return s;
}

kg_status kg_debug_time_kernel(kg_plan_t *plan, int kernel, int reps, float *ms)
{
    if (!plan || !ms || reps < 1 || kernel < 0 || kernel > 3) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    hipEvent_t e0, e1;
    HIPCHK(plan, hipEventCreate(&e0));
    HIPCHK(plan, hipEventCreate(&e1));
    void *Sc, *Sp;
    step_levels(p, p.steps, Sc, Sp);
    auto launch = [&]() {
        switch (kernel) {
        case 0: p.ops->x(p, X_STEP, nullptr, nullptr, p.chi); break;
        case 1: p.ops->y(p, -1, true); break;
        case 2: p.ops->z(p, Z_STEP, Sp, Sc, p.invM, 0); break;
        case 3: p.ops->y(p, 1, true); break;
        }
    };
    launch();  // warm-up
    HIPCHK(plan, hipEventRecord(e0, p.stream));
    for (int i = 0; i < reps; ++i) launch();
    HIPCHK(plan, hipEventRecord(e1, p.stream));
    LAUNCHCHK(plan);
    HIPCHK(plan, hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(plan, hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.ready = false;  // the time levels no longer form a valid pair
    return KG_OK;
}

kg_status kg_debug_scale_mode(kg_plan_t *plan, int kx, int ky, int kz, double factor)
{
    if (!plan) return KG_E_INVALID;
    Plan &p = P(plan);
    if (!p.ready) return fail(plan, KG_E_INVALID, "kg_set_state has not been called");
    if (kx < 0 || kx >= p.H || ky < 0 || ky >= p.n || kz < 0 || kz >= p.n || !std::isfinite(factor))
        return fail(plan, KG_E_INVALID, "mode index or factor out of range");
    Ctl c;
    kg_status s = read_ctl(plan, c);
    if (s != KG_OK) return s;
    if (c.flag) return stop_status(c);
    // the state layout [ky][kx tile][kz][kx within the tile]
    const size_t off = (size_t)((((long)ky * p.ntx + kx / p.W) * p.n + kz) * p.W + kx % p.W) * p.esz;
    if (increment(p)) {
        // FP32: S[0] = v^n, S[1] = Delta^n = v^n - v^{n-1}; v^{n-1} is kept
        float v[2], d[2];
        HIPCHK(plan, hipMemcpy(v, p.S[0] + off, sizeof v, hipMemcpyDeviceToHost));
        HIPCHK(plan, hipMemcpy(d, p.S[1] + off, sizeof d, hipMemcpyDeviceToHost));
        for (int i = 0; i < 2; ++i) {
            const double old = v[i];
            v[i] = (float)(factor * old);
            d[i] = (float)((double)d[i] + ((double)v[i] - old));
        }
        HIPCHK(plan, hipMemcpy(p.S[0] + off, v, sizeof v, hipMemcpyHostToDevice));
        HIPCHK(plan, hipMemcpy(p.S[1] + off, d, sizeof d, hipMemcpyHostToDevice));
    } else {
        double v[2];
        char *S = p.S[c.step & 1];
        HIPCHK(plan, hipMemcpy(v, S + off, sizeof v, hipMemcpyDeviceToHost));
        v[0] *= factor;
        v[1] *= factor;
        HIPCHK(plan, hipMemcpy(S + off, v, sizeof v, hipMemcpyHostToDevice));
    }
    // the resting field of the changed level, which the next step starts from
    const void *Sc, *Ssub;
    stored_level(p, c, 0, Sc, Ssub);
    if ((s = prepare_q(plan, Sc, Ssub)) != KG_OK) return s;
    HIPCHK(plan, hipStreamSynchronize(p.stream));
    return KG_OK;
}

kg_status kg_debug_copy(void *d_dst, const void *d_src, size_t bytes, int reps, void *hip_stream,
                        float *ms)
{
    if (!d_dst || !d_src || bytes % 16 || reps < 1 || !ms) return KG_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KG_E_HIP;
    const long n16 = (long)(bytes / 16);
    const unsigned grid = 256 * 128;
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, (uint4 *)d_dst, (const uint4 *)d_src, n16);
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i)
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, (uint4 *)d_dst, (const uint4 *)d_src, n16);
    (void)hipEventRecord(e1, st);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return KG_E_HIP;
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return KG_OK;
}

double kg_kernel_bytes(const kg_plan_t *plan, int kernel)
{
    if (!plan || kernel < 0 || kernel > 3) return 0.0;
    // one sweep = every half-spectrum value once
    const double sweep = (double)plan->n * plan->n * plan->H * (double)plan->esz;
    const double zsweeps = plan->p.precision == KG_FP32 ? 6.0 : 5.0;  // + Delta read/write
    return kernel == 2 ? zsweeps * sweep : 2.0 * sweep;
}

}  // extern "C"
