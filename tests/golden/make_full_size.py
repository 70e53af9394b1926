"""Write the oracle's reference values for the full-size parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``kg_inputs``): nothing here touches the GPU library.  Each case is one run
of the second-order scheme of Sec. 1.1.2, eq. (2), for the real cubic
Klein-Gordon equation (Sec. 1, eq. (1)) on the box [-4 pi, 4 pi)^3 from the
Gaussian u(0) = A exp(-(x^2/sx^2 + y^2/sy^2 + z^2/sz^2)), u_t(0) = 0.

Field cases (``field_<n>_A<A>.npz``), per stored level m (100, and 200 or
500 where listed): the physical field u^m on a strided 32^3 subsample
``u[::n/32, ::n/32, ::n/32]`` and on the central 16^3 block
``u[n/2-8:n/2+8]`` (all three axes), and the L2 norm of the whole field;
per level 0..last: the energy E^{m-1/2} of Sec. 1.1 (index m), max|u^m| and
Q4^m = h^3 sum (u^m)^4.  Runs longer than 100 steps go in segments of 100
steps, each started from the two-level restart (u^{m-1}, u^m) of the one
before, which reproduces a straight run to rounding (measured at 32^3,
A = 1.5, 300 steps: 3e-14 relative at worst; tests/test_golden_script.py) and
bounds the memory a segment's output holds.

Sweep cases (``batch_cases.json``): runs of the batched sweep's sizes (96^3,
128^3) with the blow-up test max|u| > 1e3; per run the blow-up level (-1 if
none), E^{-1/2}, the final energy, the largest max|u| over the levels
computed, and the same run from data scaled by (1 + 1e-13), which measures
how strongly the run amplifies a relative perturbation near its blow-up.

Usage: ``python tests/golden/make_full_size.py [field|batch|all] [--only NAME]``.
512^3 needs about 10 GB of host memory and roughly 13 s per step on 8 cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import kg_inputs as ki  # noqa: E402
import oracle  # noqa: E402

DT = 0.005
THRESHOLD = 1e3

# (n, A, sigma, stored levels)
FIELD_CASES = [
    (256, 1.5, (1.0, 1.0, 1.0), (100, 200)),
    (384, 0.1, (1.0, 1.0, 1.0), (100,)),
    (384, 1.5, (1.0, 1.0, 1.0), (100,)),
    (512, 0.1, (1.0, 1.0, 1.0), (100, 500)),
    (512, 1.5, (1.0, 1.0, 1.0), (100, 200)),
]

BATCH_CASES = [
    dict(n=96, A=3.0, sigma=(1.2, 0.9, 1.5), max_steps=400),
    dict(n=96, A=1.0, sigma=(0.8, 1.3, 1.0), max_steps=200),
    dict(n=128, A=3.5, sigma=(1.0, 1.4, 1.1), max_steps=300),
    dict(n=128, A=1.4, sigma=(1.1, 0.7, 0.9), max_steps=150),
]


def field_name(n, A):
    return f"field_{n}_A{A:g}.npz"


def samples(u):
    n = u.shape[0]
    s = n // 32
    c = n // 2
    return (np.ascontiguousarray(u[::s, ::s, ::s]),
            np.ascontiguousarray(u[c - 8:c + 8, c - 8:c + 8, c - 8:c + 8]),
            float(np.linalg.norm(u)))


def make_field(n, A, sigma, levels):
    t0 = time.time()
    u0 = ki.gaussian(n, A, sigma)
    out = dict(n=n, A=A, sigma=np.array(sigma), dt=DT, levels=np.array(levels))
    energy, maxu, q4 = [], [], []
    r = oracle.run(u0, DT, 100, threshold=THRESHOLD)
    del u0
    assert r["blowup_step"] < 0, "reference run blew up"
    energy += list(r["energy"])
    maxu += list(r["maxu"])
    q4 += list(r["q4"])
    sub, blk, nrm = samples(r["u"])
    out.update(u100_sub=sub, u100_center=blk, u100_norm=nrm)
    print(f"  {n}^3 A={A}: 100 steps in {time.time() - t0:.0f} s", flush=True)
    for m in range(200, max(levels) + 1, 100):
        r = oracle.run(r["u"], DT, 100, threshold=THRESHOLD, mode=oracle.INIT_TWO_LEVEL,
                       aux=r["u_prev"])
        assert r["blowup_step"] < 0, "reference run blew up"
        # level 0 of a restart is the last level of the segment before
        energy += list(r["energy"][1:])
        maxu += list(r["maxu"][1:])
        q4 += list(r["q4"][1:])
        if m in levels:
            sub, blk, nrm = samples(r["u"])
            out.update({f"u{m}_sub": sub, f"u{m}_center": blk, f"u{m}_norm": nrm})
        print(f"  {n}^3 A={A}: {m} steps in {time.time() - t0:.0f} s", flush=True)
    out.update(energy=np.array(energy), maxu=np.array(maxu), q4=np.array(q4),
               oracle_threads=oracle.num_threads())
    path = os.path.join(HERE, field_name(n, A))
    np.savez(path, **out)
    print(f"wrote {path}", flush=True)


def summarize(r, max_steps):
    b = r["blowup_step"]
    last = b if b >= 0 else max_steps
    return dict(blowup_step=int(b), E0=float(r["energy"][0]),
                E_final=None if b >= 0 else float(r["energy"][max_steps]),
                max_abs_u=float(np.max(r["maxu"][:last + 1])))


def make_batch():
    out = []
    for c in BATCH_CASES:
        t0 = time.time()
        u0 = ki.gaussian(c["n"], c["A"], c["sigma"])
        ref = summarize(oracle.run(u0, DT, c["max_steps"], threshold=THRESHOLD), c["max_steps"])
        pert = summarize(oracle.run(u0 * (1 + 1e-13), DT, c["max_steps"], threshold=THRESHOLD),
                         c["max_steps"])
        out.append(dict(c, sigma=list(c["sigma"]), dt=DT, threshold=THRESHOLD, ref=ref,
                        perturbed_1e13=pert))
        print(f"  batch {c}: {ref} ({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(HERE, "batch_cases.json")
    with open(path, "w") as f:
        json.dump(dict(oracle_threads=oracle.num_threads(), cases=out), f, indent=1)
    print(f"wrote {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="?", default="all", choices=("field", "batch", "all"))
    ap.add_argument("--only", default=None, help="one field file name, e.g. field_256_A1.5.npz")
    a = ap.parse_args()
    if a.what in ("batch", "all"):
        make_batch()
    if a.what in ("field", "all"):
        for n, A, sigma, levels in FIELD_CASES:
            if a.only and a.only != field_name(n, A):
                continue
            make_field(n, A, sigma, levels)


if __name__ == "__main__":
    main()
