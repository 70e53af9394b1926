"""Benchmark: time steps per second of the 512^3 FP64 Klein-Gordon stepper.

Workload: 512^3 real grid on the periodic box [-4 pi, 4 pi)^3, Gaussian
u0 = 0.1 exp(-(x^2 + y^2 + z^2)), u_t0 = 0, dt = 0.005, FP64, scheme of
eq. (2).  A step is one pass of the whole hot path: slab by slab of z planes
the inverse y pass, the x pass with the cubic term and the forward y pass,
then the z pass with the update and energy, then the finalize.  The initial
field is resident in HBM before timing starts.

Prints one JSON line.  Also reports the dominant kernel's roofline figures
(its algorithmic bytes over its average launch time, measured with HIP
events inside the timed steps) and the CPU oracle timed on a bounded sample
(three 512^3 steps) on this host.  Secondary legs: the FP32 path, a complex
field (u0 times the phase exp(i x / 2), cubic term |u|^2 u) in both
precisions, and the batched parametric sweep.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--amplitude", type=float, default=0.1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--energy-every", type=int, default=50)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-runs", type=int, default=512)
    ap.add_argument("--sweep-seq-sample", type=int, default=16)
    ap.add_argument("--complex", choices=("on", "off", "only"), default="on",
                    help="complex-field legs: with the real ones (on), none (off), or alone "
                         "(only: one JSON line for the complex FP64 leg, for profiling)")
    return ap.parse_args()


def sweep(args, kg, ki, torch):
    """Batched parametric sweep: seeded runs over grid sizes {48, 64, 96, 128},
    A ~ U[0.5, 4], sigma ~ U[0.5, 2] per axis, dt = 0.005, up to 2000 steps or
    blow-up (max|u| > 1e3), against a sequential kg_step loop on a sample."""
    import numpy as np
    draws = ki.sweep_runs(args.sweep_runs, seed=0)
    runs = [dict(n=d["n"], A=d["A"], sigma=d["sigma"], dt=0.005, max_steps=2000, threshold=1e3)
            for d in draws]
    cache = os.environ.get("KG_TUNE_CACHE",
                           os.path.join(ROOT, "paper_1501_04552_amd", "tune_cache.json"))
    res, secs = kg.kg_batch_run(runs, tune=True, tune_cache=cache)
    steps = sum(r["steps_done"] for r in res)
    sweep_bytes = sum(11 * r["n"] ** 2 * (r["n"] // 2 + 1) * 16 * o["steps_done"]
                      for r, o in zip(runs, res))
    # sequential reference: the same runs one by one through kg_step (sample)
    sample = runs[:args.sweep_seq_sample]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_blown = []
    for r in sample:
        with kg.Solver(r["n"], r["dt"], blowup_threshold=r["threshold"]) as s:
            s.set_state(torch.from_numpy(ki.gaussian(r["n"], r["A"], r["sigma"])).cuda())
            st, done = s.step(r["max_steps"])
            seq_blown.append(s.stats()[1])
    torch.cuda.synchronize()
    seq_secs = time.perf_counter() - t0
    agree = sum(int(b == o["blew_up"]) for b, o in zip(seq_blown, res))
    return {"workload": f"{len(runs)} runs, seed 0, n in {{48,64,96,128}}, A~U[0.5,4], "
                        "sigma~U[0.5,2], dt=0.005, <=2000 steps, blow-up at max|u|>1e3, FP64",
            "seconds": secs, "runs_per_hour": len(runs) / secs * 3600.0,
            "run_steps_per_s": steps / secs, "blown_fraction": float(np.mean([o["blew_up"] for o in res])),
            "model_GBs": sweep_bytes / secs / 1e9,
            "sequential_kg_step": {"runs": len(sample), "seconds_incl_setup": seq_secs,
                                   "runs_per_hour": len(sample) / seq_secs * 3600.0,
                                   "labels_agree": agree}}


def traffic_from_profiles(n):
    """Counter-derived HBM bytes per launch of the z pass, if a committed
    measurement for this grid size exists (profiles/*counters*.json)."""
    path = os.path.join(ROOT, "profiles", f"z_update_{n}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("source_hash") != kernel_source_hash():
            return None
        return d.get("bytes_per_launch")
    except Exception:
        return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kg_fft.hpp", "kg_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1501_04552_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(u0, dt, steps=3):
    """The oracle on this host: a few steps of the same workload (set-up
    excluded; about 12 s at 512^3 on 16 threads)."""
    import oracle
    r = oracle.run(u0, dt, steps)
    secs = r["loop_seconds"]
    return {"value": steps / secs if secs > 0 else None, "unit": "steps/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} time steps of the {u0.shape[0]}^3 FP64 workload (set-up "
                      f"excluded), {secs:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this solver keeps the "
              "whole grid on a single device and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import kg_inputs as ki
    import paper_1501_04552_amd as kg

    torch.cuda.set_device(0)
    n, dt = args.n, args.dt
    u0 = ki.gaussian(n, args.amplitude)
    u0_dev = torch.from_numpy(u0).cuda()

    def timed_run(precision, complex_field=False):
        """Warm up, time args.steps steps (graph replays), then an event-timed
        run of the same length for per-kernel durations."""
        solver = kg.Solver(n, dt, blowup_threshold=1e3, precision=precision,
                           complex_field=complex_field)
        if complex_field:
            x = torch.from_numpy(ki.axis(n)).cuda()
            solver.set_state((u0_dev.to(torch.complex128) * torch.exp(0.5j * x)).contiguous())
        else:
            solver.set_state(u0_dev)
        E0, _ = solver.energy()
        solver.step(args.warmup, sync=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kg.kg_step(solver.plan, args.steps, 0)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        done, blown, _ = solver.stats()
        if blown:
            raise RuntimeError("the benchmark run blew up")
        elin, q4, _ = solver.records(0, done)
        series = [(m, float(elin[m] - (q4[m] + q4[m + 1]) / 8.0))
                  for m in range(0, done - 1, args.energy_every)]
        E_end, _ = solver.energy()
        kg.kg_step(solver.plan, args.steps, kg.KG_STEP_TIMED)
        ms, _ = kg.kg_kernel_times(solver.plan)
        kbytes = [kg.kg_kernel_bytes(solver.plan, i) for i in range(4)]
        solver.close()
        return dict(elapsed=elapsed, series=series, drift=abs(E_end - E0) / abs(E0), ms=ms,
                    kbytes=kbytes)

    def complex_legs():
        out = {}
        for name, prec in (("fp32", kg.KG_FP32), ("fp64", kg.KG_FP64)):
            torch.cuda.empty_cache()
            out[name] = complex_leg(prec)
        torch.cuda.empty_cache()
        return dict(out, workload=f"KG {n}^3 complex u0 = {args.amplitude} exp(-|x|^2) "
                                  f"exp(i x/2), u_t0 = 0, |u|^2 u, dt={dt}; full spectrum per level")

    def complex_leg(prec):
        rc = timed_run(prec, complex_field=True)
        tc = rc["elapsed"] / args.steps
        zc = rc["kbytes"][kg.KERNELS.index("z_update")] / (rc["ms"][2] * 1e-3) / 1e9
        sweep_c = n ** 3 * (16 if prec == kg.KG_FP64 else 8)  # full spectrum, one pass
        return {"steps_per_s": 1.0 / tc, "ms_per_step": 1e3 * tc,
                "kernels_ms": dict(zip(kg.KERNELS, rc["ms"])),
                "z_update_GBs": zc, "z_update_hbm_frac": zc / HBM_PEAK_GBS,
                "step_model_GBs": (11 if prec == kg.KG_FP64 else 12) * sweep_c / tc / 1e9,
                "energy_drift": rc["drift"]}

    if args.complex == "only":
        c = complex_legs()
        print(json.dumps({"metric": f"{n}^3 complex-field time steps/s (FP64)",
                          "value": c["fp64"]["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": c["fp64"]["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": c["workload"]},
                          "complex_field": c}), flush=True)
        return
    # FP32 first: each precision's workspace is then fresh device memory, as
    # for a single solver in a new process (FP32 placed in the block freed by
    # the FP64 solver measured about 2% slower; FP64 does not depend on it)
    r32 = timed_run(kg.KG_FP32)
    r64 = timed_run(kg.KG_FP64)
    cplx = complex_legs() if args.complex == "on" else None
    for m, e in r64["series"]:
        print(f"step {m:5d}  E^(m+1/2) = {e:.15e}", file=sys.stderr)
    elapsed, drift, ms = r64["elapsed"], r64["drift"], r64["ms"]
    zi = kg.KERNELS.index("z_update")
    zbytes = r64["kbytes"][zi]
    z_gbs = zbytes / (ms[zi] * 1e-3) / 1e9
    kernels = {name: {"ms": ms[i], "GB/s": (r64["kbytes"][i] / (ms[i] * 1e-3) / 1e9
                                            if i < 4 and ms[i] > 0 else None)}
               for i, name in enumerate(kg.KERNELS)}

    # precision study: A = 1.5, sigma = 1, dt = 0.005, 200 steps, FP32 vs FP64
    ua = ki.gaussian(n, 1.5)
    res = {}
    for prec in (kg.KG_FP64, kg.KG_FP32):
        with kg.Solver(n, dt, precision=prec) as s:
            s.set_state(ua)
            Ea, _ = s.energy()
            s.step(200)
            res[prec] = (s.u(), abs(s.energy()[0] - Ea) / abs(Ea))
    rel32 = float(np.linalg.norm(res[1][0] - res[0][0]) / np.linalg.norm(res[0][0]))
    drift_a = {"fp64": res[0][1], "fp32": res[1][1]}
    del ua, res
    # achievable-bandwidth ceiling: the library's plain copy kernel, 1 GiB
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nb, dtype=torch.uint8, device="cuda")
    cms = kg.kg_debug_copy(dst.data_ptr(), src.data_ptr(), nb, 20,
                           torch.cuda.current_stream().cuda_stream)
    copy_gbs = 2 * nb / (cms * 1e-3) / 1e9
    del src, dst

    steps_per_s = args.steps / elapsed
    sweep_b = n * n * (n // 2 + 1) * 16  # one sweep of the FP64 half spectrum
    step_bytes = 11 * sweep_b
    t32 = r32["elapsed"] / args.steps
    fp32 = {"steps_per_s": 1.0 / t32, "ms_per_step": 1e3 * t32,
            "speedup_vs_fp64": (1.0 / t32) / steps_per_s,
            "step_model_GBs": 12 * sweep_b / 2 / t32 / 1e9,
            "step_hbm_frac": 12 * sweep_b / 2 / t32 / 1e9 / HBM_PEAK_GBS,
            "kernels_ms": dict(zip(kg.KERNELS, r32["ms"])),
            "energy_drift": r32["drift"],
            "precision_study": {"workload": f"{n}^3 A=1.5 sigma=1 dt={dt} 200 steps",
                                "rel_l2_fp32_vs_fp64": rel32,
                                "energy_drift_fp64": drift_a["fp64"],
                                "energy_drift_fp32": drift_a["fp32"]}}
    line = {
        "metric": "512^3 time steps/s (FP64)" if n == 512 else f"{n}^3 time steps/s (FP64)",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"KG {n}^3 FP64 Gaussian A={args.amplitude} sigma=1 "
                               f"box [-4pi,4pi)^3 dt={dt}", "grid": n, "dt": dt,
                   "precision": "fp64"},
        "roofline": {"bound": "hbm", "kernel": "z_update", "achieved": z_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": z_gbs / HBM_PEAK_GBS,
                     "traffic": traffic_from_profiles(n),
                     "algorithmic_bytes_per_launch": zbytes, "avg_launch_ms": ms[zi]},
        "step_model_GBs": step_bytes / (elapsed / args.steps) / 1e9,
        "step_hbm_frac": step_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS,
        "step_model_note": "11 algorithmic sweeps of the half spectrum per step over the step "
                           "time; the y-inverse / x / y-forward chain runs in slabs that the "
                           "256 MB memory-side cache serves in part, so this is an effective "
                           "rate, not HBM traffic",
        "kernels": kernels,
        "copy_GBs": copy_gbs,
        "energy_drift": drift,
        "fp32": fp32,
    }
    if cplx:
        line["complex_field"] = cplx
    if not args.no_sweep:
        line["sweep"] = sweep(args, kg, ki, torch)
    if not args.no_cpu_baseline and n <= 512:
        line["cpu_baseline"] = cpu_baseline(u0, dt)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
