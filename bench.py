"""Benchmark: time steps per second of the 512^3 FP64 Klein-Gordon stepper.

Workload: 512^3 real grid on the periodic box [-4 pi, 4 pi)^3, Gaussian
u0 = 0.1 exp(-(x^2 + y^2 + z^2)), u_t0 = 0, dt = 0.005, FP64, scheme of
eq. (2).  A step is one pass of the whole hot path: slab by slab of z planes
the inverse y pass, the x pass with the cubic term and the forward y pass,
then the z pass with the update and energy, then the finalize.  The initial
field is resident in HBM before timing starts.

Prints one JSON line.  `value` = steps / wall time of exactly --steps steps
bracketed by device synchronisations, after --warmup untimed steps; the step
graphs are captured when the state is set, so no capture or set-up falls in
the timed region.  Also reported: the median over 5 repetitions of a 50-step
run timed by HIP events on the solver's stream; the dominant kernel's
roofline figures (its algorithmic bytes over its average launch time,
measured with HIP events); and the CPU oracle, built for this host, timed on
a bounded sample on this host's cores (all threads, and one thread).
Secondary legs: the FP32 path, the precision study against the oracle's
reference fields, a complex field (u0 times the phase exp(i x / 2), cubic
term |u|^2 u) in both precisions, the batched parametric sweep and the
blow-up surrogate.
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
    ap.add_argument("--surrogate", choices=("off", "small", "full"), default="small",
                    help="surrogate leg: off, small (2048 training / 512 held-out runs), or "
                         "full (8192 / 1024 runs)")
    ap.add_argument("--event-reps", type=int, default=5)
    ap.add_argument("--event-steps", type=int, default=50)
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
    with open(cache) as f:
        tuned = json.load(f)
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
            "tuned": {k: v for k, v in sorted(tuned.items())
                      if int(k.split("/")[1]) in ki.SWEEP_SIZES},
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


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def native_oracle():
    """Path of the oracle compiled for this host (-O3 -march=native -fopenmp)."""
    import tempfile
    from oracle.build import build_oracle
    d = tempfile.mkdtemp(prefix="kg_oracle_native_")
    return build_oracle(out=os.path.join(d, "libkg_oracle_native.so"),
                        opt=("-O3", "-march=native"))


ONE_THREAD_CODE = """
import json, sys
sys.path.insert(0, {root!r})
import oracle, kg_inputs as ki
o = oracle.Oracle({lib!r})
r = o.run(ki.gaussian({n}, {A}), {dt}, {steps})
print(json.dumps({{"seconds": r["loop_seconds"], "threads": o.num_threads()}}))
"""


def start_one_thread_baseline(lib, n, A, dt, steps=1):
    """The oracle on one host thread, in a child process (its set-up alone
    takes about a minute at 512^3, so it runs while the GPU legs do)."""
    import subprocess
    code = ONE_THREAD_CODE.format(root=ROOT, lib=lib, n=n, A=A, dt=dt, steps=steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE,
                            stderr=subprocess.PIPE, text=True)


def cpu_baseline(lib, u0, dt, one_thread, steps=5):
    """The oracle on this host's cores: `steps` steps of the same workload on
    all threads (set-up excluded), plus the one-thread child's result."""
    import oracle
    o = oracle.Oracle(lib)
    r = o.run(u0, dt, steps)
    secs = r["loop_seconds"]
    out = {"value": steps / secs if secs > 0 else None, "unit": "steps/s",
           "cores": o.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
           "build": "gcc -O3 -march=native -fopenmp on this host",
           "sample": f"{steps} time steps of the {u0.shape[0]}^3 FP64 workload (set-up "
                     f"excluded), {secs:.2f} s on {o.num_threads()} threads"}
    if one_thread is not None:
        so, se = one_thread.communicate(timeout=900)
        if one_thread.returncode == 0:
            d = json.loads(so.strip().splitlines()[-1])
            out["one_thread"] = {"value": 1.0 / d["seconds"], "unit": "steps/s",
                                 "threads": d["threads"],
                                 "sample": f"1 time step of the same workload, "
                                           f"{d['seconds']:.1f} s"}
        else:
            out["one_thread"] = {"error": se[-500:]}
    return out


def golden_compare(kg, ki, np, torch, n, A, steps=200):
    """The precision workload (A = 1.5, sigma = 1, dt = 0.005, 200 steps) in
    both precisions, each against the oracle's reference field and energies
    (tests/golden/field_<n>_A1.5.npz, written from oracle/ only): relative
    L2 over the stored samples (strided 32^3 and central 16^3) and the energy
    drift of the run."""
    path = os.path.join(ROOT, "tests", "golden", f"field_{n}_A{A:g}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    out = {"workload": f"{n}^3 A={A} sigma=1 dt={float(g['dt'])} {steps} steps; u compared on "
                       "a strided 32^3 subsample and the central 16^3 block",
           "energy_drift_oracle": float(abs(g["energy"][steps] - g["energy"][0]) /
                                        abs(g["energy"][0]))}
    for name, prec in (("fp64", kg.KG_FP64), ("fp32", kg.KG_FP32)):
        with kg.Solver(n, float(g["dt"]), precision=prec) as s:
            s.set_state(torch.from_numpy(ki.gaussian(n, A)).cuda())
            s.step(steps)
            u = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
            s.u(u)
            st, c = n // 32, n // 2
            got = np.concatenate([u[::st, ::st, ::st].cpu().numpy().ravel(),
                                  u[c - 8:c + 8, c - 8:c + 8, c - 8:c + 8].cpu().numpy().ravel()])
            del u
            E = s.energies(0, steps + 1)
        ref = np.concatenate([g[f"u{steps}_sub"].ravel(), g[f"u{steps}_center"].ravel()])
        out[name] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                     "energy_max_rel_diff_vs_oracle":
                         float(np.max(np.abs(E - g["energy"][:steps + 1]) /
                                      np.abs(g["energy"][:steps + 1]))),
                     "energy_drift": float(abs(E[-1] - E[0]) / abs(E[0]))}
    return out


def pcie_inclusive(torch, u0, elapsed, steps):
    """The rate when the initial field comes from host memory and u of the
    last level goes back to it: the timed steps plus one host-to-device and
    one device-to-host copy of a real field (pageable numpy memory, as a
    caller's arrays would be).  A note beside `value`, never `value`."""
    reps = 3
    t_h2d = t_d2h = 1e30
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = torch.from_numpy(u0).cuda()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h = d.cpu()
        t2 = time.perf_counter()
        t_h2d, t_d2h = min(t_h2d, t1 - t0), min(t_d2h, t2 - t1)
        del d, h
    total = elapsed + t_h2d + t_d2h
    return {"steps_per_s": steps / total, "h2d_seconds": t_h2d, "d2h_seconds": t_d2h,
            "field_GB": u0.nbytes / 1e9,
            "note": f"{steps} timed steps plus one {u0.nbytes / 1e9:.2f} GB field each way over "
                    "PCIe (best of 3 copies each)"}


def energy_vs_oracle(np, n, A, dt, series):
    """The timed run's energy series E^{m-1/2} (every --energy-every levels)
    against the oracle's run of the same workload (tests/golden/field_<n>_A<A>.npz,
    written from oracle/ only), at the levels both have."""
    path = os.path.join(ROOT, "tests", "golden", f"field_{n}_A{A:g}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    if abs(float(g["dt"]) - dt) > 1e-15 or np.any(np.asarray(g["sigma"]) != 1.0):
        return None
    ref = g["energy"]
    pts = [(m, e) for m, e in series if m < len(ref)]
    if not pts:
        return None
    rel = [abs(e - ref[m]) / abs(ref[m]) for m, e in pts]
    return {"levels": [m for m, _ in pts], "max_rel_diff": float(max(rel)),
            "oracle_levels": int(len(ref) - 1)}


def surrogate_leg(mode):
    """The blow-up surrogate on the sweep distribution at 64^3: solver labels,
    training by the library's kernels, held-out accuracy with solver fallback,
    and the cost of building it (labelling + training) against the time it
    saves per query (break-even query count)."""
    from paper_1501_04552_amd import surrogate as sg
    ntr, nte = (8192, 1024) if mode == "full" else (2048, 512)
    return sg.main(["--train", str(ntr), "--test", str(nte), "--quiet"])


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
        """Warm up, time args.steps steps (graph replays) between device
        synchronisations, repeat a 50-step run timed by HIP events, then an
        event-per-kernel run of the same length for per-kernel durations."""
        solver = kg.Solver(n, dt, blowup_threshold=1e3, precision=precision,
                           complex_field=complex_field)
        if complex_field:
            x = torch.from_numpy(ki.axis(n)).cuda()
            solver.set_state((u0_dev.to(torch.complex128) * torch.exp(0.5j * x)).contiguous())
        else:
            solver.set_state(u0_dev)
        # set-up, outside the timed region: set_state captured and uploaded the
        # step graphs; launch each once (8-step and single-step, both level
        # parities), then start the run again from the initial data
        solver.step(2 * 8 + 2, sync=True)
        if complex_field:
            solver.set_state((u0_dev.to(torch.complex128) * torch.exp(0.5j * x)).contiguous())
        else:
            solver.set_state(u0_dev)
        solver.step(args.warmup, sync=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kg.kg_step(solver.plan, args.steps, 0)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        done, blown, _ = solver.stats()
        if blown:
            raise RuntimeError("the benchmark run blew up")
        # energy E^{m-1/2} every args.energy_every levels, through the library
        levels = list(range(0, done + 1, args.energy_every))
        if levels[-1] != done:
            levels.append(done)
        series = [(m, float(solver.energies(m, 1)[0])) for m in levels]
        drift = abs(series[-1][1] - series[0][1]) / abs(series[0][1])
        # HIP events on the solver's stream around repeated graph runs
        ev_ms = []
        for _ in range(args.event_reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(solver.stream)
            kg.kg_step(solver.plan, args.event_steps, 0)
            e1.record(solver.stream)
            e1.synchronize()
            ev_ms.append(e0.elapsed_time(e1) / args.event_steps)
        kg.kg_step(solver.plan, args.steps, kg.KG_STEP_TIMED)
        ms, _ = kg.kg_kernel_times(solver.plan)
        kbytes = [kg.kg_kernel_bytes(solver.plan, i) for i in range(4)]
        solver.close()
        return dict(elapsed=elapsed, series=series, drift=drift, ms=ms, kbytes=kbytes,
                    event_ms=float(np.median(ev_ms)), event_ms_all=ev_ms)

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
    one_thread, oracle_lib = None, None
    if not args.no_cpu_baseline and n <= 512:
        oracle_lib = native_oracle()
        one_thread = start_one_thread_baseline(oracle_lib, n, args.amplitude, dt)
    cplx = complex_legs() if args.complex == "on" else None
    for m, e in r64["series"]:
        print(f"step {m:5d}  E^(m-1/2) = {e:.15e}", file=sys.stderr)
    energy_check = energy_vs_oracle(np, n, args.amplitude, dt, r64["series"])
    pcie = pcie_inclusive(torch, u0, r64["elapsed"], args.steps)
    elapsed, drift, ms = r64["elapsed"], r64["drift"], r64["ms"]
    zi = kg.KERNELS.index("z_update")
    zbytes = r64["kbytes"][zi]
    z_gbs = zbytes / (ms[zi] * 1e-3) / 1e9
    kernels = {name: {"ms": ms[i], "GB/s": (r64["kbytes"][i] / (ms[i] * 1e-3) / 1e9
                                            if i < 4 and ms[i] > 0 else None)}
               for i, name in enumerate(kg.KERNELS)}
    z32 = r32["kbytes"][zi] / (r32["ms"][zi] * 1e-3) / 1e9

    # precision study against the oracle's reference fields (A = 1.5, 200 steps)
    precision_study = {str(m): golden_compare(kg, ki, np, torch, m, 1.5) for m in (256, n)}
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
            "event_median_ms_per_step": r32["event_ms"],
            "speedup_vs_fp64_event_median": r64["event_ms"] / r32["event_ms"],
            "step_model_GBs": 12 * sweep_b / 2 / t32 / 1e9,
            "step_hbm_frac": 12 * sweep_b / 2 / t32 / 1e9 / HBM_PEAK_GBS,
            "kernels_ms": dict(zip(kg.KERNELS, r32["ms"])),
            "kernels_ms_sum": float(sum(r32["ms"])),
            "z_update_GBs": z32, "z_update_hbm_frac": z32 / HBM_PEAK_GBS,
            "energy_drift": r32["drift"]}
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
        "event_median_ms_per_step": r64["event_ms"],
        "event_ms_per_step_reps": r64["event_ms_all"],
        "event_timing": f"median of {args.event_reps} runs of {args.event_steps} steps, HIP "
                        "events on the solver's stream",
        "step_model_GBs": step_bytes / (elapsed / args.steps) / 1e9,
        "step_hbm_frac": step_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS,
        "step_model_note": "11 algorithmic sweeps of the half spectrum per step over the step "
                           "time; the y-inverse / x / y-forward chain runs in slabs that the "
                           "256 MB memory-side cache serves in part, so this is an effective "
                           "rate, not HBM traffic",
        "kernels": kernels,
        "kernels_ms_sum": float(sum(ms)),
        "copy_GBs": copy_gbs,
        "energy_drift": drift,
        "energy_vs_oracle": energy_check,
        "pcie_inclusive": pcie,
        "fp32": fp32,
        "precision_study": precision_study,
    }
    if cplx:
        line["complex_field"] = cplx
    if not args.no_sweep:
        line["sweep"] = sweep(args, kg, ki, torch)
    if args.surrogate != "off":
        line["surrogate"] = surrogate_leg(args.surrogate)
    if oracle_lib:
        line["cpu_baseline"] = cpu_baseline(oracle_lib, u0, dt, one_thread)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
