// kg_plan.hpp -- host-side plan object and the kernel launchers per
// (precision, grid size, tile width), shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <memory>
#include <string>
#include <vector>

#include "../../include/kg.h"
#include "kg_kernels.hpp"

namespace kg {

struct Ops;

}  // namespace kg

struct kg_plan_s {
    kg_params p{};
    int n = 0, H = 0, W = 0, ntx = 0, P = 0;
    int cf = 0;   // complex field: full spectrum (H = n), cubic term |u|^2 u
    int dkc = 0;  // dealiasing cut-off n/3 of the nonlinear term, 0 when off
    long PZ = 0;  // plane pitch of Q in elements (n * P plus optional padding)
    int zslab = 0;  // z planes per slab of the y-inverse / x / y-forward chain
    double L = 0, h3 = 0, ks2 = 0, invM = 0, escale = 0, chi = 1;
    double e_tol = 0;  // energy alarm tolerance (kg_set_energy_alarm), 0 when off
    size_t esz = 16;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    bool own_ws = false;
    size_t ws_bytes = 0;
    char *Q = nullptr, *S[2] = {nullptr, nullptr}, *tw = nullptr;
    double *partA = nullptr, *partC = nullptr, *sub = nullptr;
    kg::Rec *rec = nullptr;
    kg::Ctl *ctl = nullptr;
    long nA = 0, nC = 0;
    size_t q_bytes = 0, s_bytes = 0;
    long steps = 0;  // steps launched since the state was set
    bool ready = false;
    std::unique_ptr<kg::Ops> ops;
    std::vector<hipEvent_t> tev;  // events of KG_STEP_TIMED calls
    hipStream_t cap = nullptr;    // private stream used only to capture graphs
    hipStream_t cap2 = nullptr;   // second capture stream: odd slabs of the chain
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // GRAPH_STEPS steps from parity 0 / 1
    hipGraphExec_t gexec1[2] = {nullptr, nullptr};  // one step from parity 0 / 1
    double kt_ms[5] = {0, 0, 0, 0, 0};
    int kt_steps = 0;
    std::string err;
};

namespace kg {

using Plan = kg_plan_s;

constexpr int PAIR_BLOCKS = 1024;

// Kernel launchers for one (precision, grid size, tile width).
struct Ops {
    virtual ~Ops() = default;
    // x and y launch over planes z0 .. z0+nz-1 (nz = 0 or n: all); partial
    // slabs must hold whole workgroups (multiples of slab_quantum) and apply
    // to the x pass in X_STEP / X_REDUCE only.
    virtual void x(Plan &pl, int mode, const double *rin, double *rout, double chi,
                   const double *rin2 = nullptr, int z0 = 0, int nz = 0) = 0;
    virtual void y(Plan &pl, int dir, bool check_flag, int z0 = 0, int nz = 0) = 0;
    virtual void z(Plan &pl, int mode, void *Sp, void *Sc, double scale, int has_vel,
                   const void *Ssub = nullptr) = 0;
    virtual void pair_energy(Plan &pl, const void *S0, const void *S1) = 0;
    virtual void state_to_spec(Plan &pl, const void *S, const void *Ssub, double *out) = 0;
    virtual void q_to_spec(Plan &pl, double *out) = 0;
    virtual void spec_to_q(Plan &pl, const double *in) = 0;
    virtual long x_blocks(int cf) const = 0;
    virtual long z_blocks(int ntx) const = 0;
    virtual long z_step_parts(int ntx) const = 0;  // energy partials a Z_STEP writes
    virtual int slab_quantum() const = 0;  // slab sizes must be multiples of this
};

// Launchers of one precision (defined in kg_ops_f64.hip / kg_ops_f32.hip).
std::unique_ptr<Ops> make_ops_f64(int n, int W);
std::unique_ptr<Ops> make_ops_f32(int n, int W);

// Whether the persistent z pass also prefetches the next tile's Q values
// (besides its state): at 512^3 FP32 with the prefetch 0.643 against 0.658
// ms, FP64 without it 1.013 against 1.085 ms (its 172 registers grow to 204).
template <typename T>
constexpr int zstep_prefetch() { return sizeof(T) == 4 ? 1 : 0; }

// Persistent workgroups of the step's z pass (k_zstep): as many as the
// device holds at once (0: the tile kernel k_zpass runs instead, as it does
// when KG_Z_PERSISTENT=0).
template <typename T, int N, int W>
int zstep_slots()
{
    if (const char *e = std::getenv("KG_Z_PERSISTENT"))
        if (std::atoi(e) == 0) return 0;
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_zstep<T, N, W, zstep_prefetch<T>()>,
                                                     YZCfg<N, W>::NT, 0) !=
            hipSuccess)
        return 0;
    return cus * occ;
}

template <typename T, int N, int W>
struct OpsImpl final : Ops {
    using YC = YZCfg<N, W>;
    static long yz_grid(int ntx) { return (long)ntx * ((N + YC::B - 1) / YC::B); }
    const int zslots = zstep_slots<T, N, W>();
    long zstep_grid(int ntx) const
    {
        const long nb = yz_grid(ntx);
        return zslots > 0 && zslots < nb ? zslots : nb;
    }

    long x_blocks(int cf) const override { return cf ? XCfg<T, N>::blocks_c() : XCfg<T, N>::blocks(); }
    long z_blocks(int ntx) const override { return yz_grid(ntx); }
    long z_step_parts(int ntx) const override { return zslots > 0 ? zstep_grid(ntx) : yz_grid(ntx); }
    int slab_quantum() const override
    {
        constexpr int ppb = XCfg<T, N>::PPB, b = YC::B;
        return ppb > b ? ppb : b;  // whole x workgroups and whole y workgroups
    }

    void x(Plan &pl, int mode, const double *rin, double *rout, double chi,
           const double *rin2, int z0, int nz) override
    {
        XArgs<T> a{};
        a.Q = (cx<T> *)pl.Q;
        a.tw = (const cx<T> *)pl.tw;
        a.rin = rin;
        a.rin2 = rin2;
        a.rout = rout;
        a.part = pl.partA;
        a.ctl = pl.ctl;
        a.P = pl.P;
        a.PZ = pl.PZ;
        a.chi = (T)chi;
        long nb = x_blocks(pl.cf);
        if (nz > 0 && nz < N && (mode == X_STEP || mode == X_REDUCE)) {
            // lines per plane: N/2 pairs of a real field, N rows of a complex one
            const long lpp = pl.cf ? N : N / 2;
            const long b0 = (long)z0 * lpp / XCfg<T, N>::PPB;
            nb = (long)nz * lpp / XCfg<T, N>::PPB;
            a.Q += (long)z0 * pl.PZ;
            a.part += 2 * b0;
        }
        dim3 g((unsigned)nb), b(256);
        if (pl.cf) {
            switch (mode) {
            case X_STEP: hipLaunchKernelGGL((k_xpass<T, N, X_STEP, true>), g, b, 0, pl.stream, a); break;
            case X_REDUCE: hipLaunchKernelGGL((k_xpass<T, N, X_REDUCE, true>), g, b, 0, pl.stream, a); break;
            case X_R2C: hipLaunchKernelGGL((k_xpass<T, N, X_R2C, true>), g, b, 0, pl.stream, a); break;
            case X_C2R: hipLaunchKernelGGL((k_xpass<T, N, X_C2R, true>), g, b, 0, pl.stream, a); break;
            }
            return;
        }
        switch (mode) {
        case X_STEP: hipLaunchKernelGGL((k_xpass<T, N, X_STEP>), g, b, 0, pl.stream, a); break;
        case X_REDUCE: hipLaunchKernelGGL((k_xpass<T, N, X_REDUCE>), g, b, 0, pl.stream, a); break;
        case X_R2C: hipLaunchKernelGGL((k_xpass<T, N, X_R2C>), g, b, 0, pl.stream, a); break;
        case X_C2R: hipLaunchKernelGGL((k_xpass<T, N, X_C2R>), g, b, 0, pl.stream, a); break;
        }
    }
    void y(Plan &pl, int dir, bool check_flag, int z0, int nz) override
    {
        YArgs<T> a{};
        a.Q = (cx<T> *)pl.Q;
        a.tw = (const cx<T> *)pl.tw;
        a.ctl = check_flag ? pl.ctl : nullptr;
        a.P = pl.P;
        a.PZ = pl.PZ;
        a.H = pl.H;
        a.ntx = pl.ntx;
        long nb = yz_grid(pl.ntx);
        if (nz > 0 && nz < N) {
            a.Q += (long)z0 * pl.PZ;
            nb = (long)pl.ntx * ((nz + YC::B - 1) / YC::B);
        }
        dim3 g((unsigned)nb), b(YC::NT);
        if (dir < 0)
            hipLaunchKernelGGL((k_ypass<T, N, W, -1>), g, b, 0, pl.stream, a);
        else
            hipLaunchKernelGGL((k_ypass<T, N, W, 1>), g, b, 0, pl.stream, a);
    }
    void z(Plan &pl, int mode, void *Sp, void *Sc, double scale, int has_vel,
           const void *Ssub) override
    {
        ZArgs<T> a{};
        a.Q = (cx<T> *)pl.Q;
        a.tw = (const cx<T> *)pl.tw;
        a.Sp = (cx<T> *)Sp;
        a.Sc = (cx<T> *)Sc;
        a.Ssub = (const cx<T> *)Ssub;
        a.part = pl.partC;
        a.ctl = pl.ctl;
        a.P = pl.P;
        a.PZ = pl.PZ;
        a.H = pl.H;
        a.ntx = pl.ntx;
        a.ks2 = pl.ks2;
        a.dt = pl.p.dt;
        a.chi = pl.chi;
        a.scale = scale;
        a.has_vel = has_vel;
        a.cf = pl.cf;
        a.dkc = pl.dkc;
        dim3 g((unsigned)yz_grid(pl.ntx)), b(YC::NT);
        switch (mode) {
        case Z_STEP:
            if (zslots > 0)
                hipLaunchKernelGGL((k_zstep<T, N, W, zstep_prefetch<T>()>), dim3((unsigned)zstep_grid(pl.ntx)),
                                   b, 0, pl.stream, a, (int)yz_grid(pl.ntx));
            else
                hipLaunchKernelGGL((k_zpass<T, N, W, Z_STEP>), g, b, 0, pl.stream, a);
            break;
        case Z_FWD_STATE: hipLaunchKernelGGL((k_zpass<T, N, W, Z_FWD_STATE>), g, b, 0, pl.stream, a); break;
        case Z_FWD_Q: hipLaunchKernelGGL((k_zpass<T, N, W, Z_FWD_Q>), g, b, 0, pl.stream, a); break;
        case Z_INV_STATE: hipLaunchKernelGGL((k_zpass<T, N, W, Z_INV_STATE>), g, b, 0, pl.stream, a); break;
        case Z_INV_Q: hipLaunchKernelGGL((k_zpass<T, N, W, Z_INV_Q>), g, b, 0, pl.stream, a); break;
        case Z_START: hipLaunchKernelGGL((k_zpass<T, N, W, Z_START>), g, b, 0, pl.stream, a); break;
        }
    }
    void pair_energy(Plan &pl, const void *S0, const void *S1) override
    {
        hipLaunchKernelGGL((k_pair_energy<T, N, W>), dim3(PAIR_BLOCKS), dim3(256), 0, pl.stream,
                           (const cx<T> *)S0, (const cx<T> *)S1, pl.partC, pl.H, pl.ntx, pl.ks2,
                           pl.p.dt, pl.cf);
    }
    void state_to_spec(Plan &pl, const void *S, const void *Ssub, double *out) override
    {
        hipLaunchKernelGGL((k_state_to_spec<T, N, W>), dim3(2048), dim3(256), 0, pl.stream,
                           (const cx<T> *)S, (const cx<T> *)Ssub, out, pl.H, pl.ntx);
    }
    void q_to_spec(Plan &pl, double *out) override
    {
        hipLaunchKernelGGL((k_q_to_spec<T>), dim3(2048), dim3(256), 0, pl.stream,
                           (const cx<T> *)pl.Q, out, pl.P, pl.PZ, N, pl.H, (long)N * N);
    }
    void spec_to_q(Plan &pl, const double *in) override
    {
        hipLaunchKernelGGL((k_spec_to_q<T>), dim3(2048), dim3(256), 0, pl.stream, in,
                           (cx<T> *)pl.Q, pl.P, pl.PZ, N, pl.H, (long)N * N);
    }
};

}  // namespace kg
