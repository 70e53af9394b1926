"""Batched parametric sweep (kg_batch_run): every run of a mixed-size batch
must reproduce the same run done alone through kg_step, and runs must not
affect each other.

Tolerances: a batched run and a single run use the same kernels and the same
per-column FFT arithmetic; only the Gaussian sampling (the library's exp on
the GPU versus numpy's on the host, 1 ulp apart) and the order of the energy
partial sums differ, so energies agree to ~1e-13 relative; 1e-11 is used.
"""
import json
import os

import numpy as np
import pytest

import kg_inputs as ki
import oracle

pytestmark = pytest.mark.gpu

RUNS = [
    dict(n=32, A=0.8, sigma=(1.0, 1.2, 0.9), dt=0.01, max_steps=120, threshold=1e3),
    dict(n=48, A=3.5, sigma=(1.0, 1.0, 1.0), dt=0.005, max_steps=400, threshold=1e3),
    dict(n=64, A=1.5, sigma=(0.7, 1.4, 1.1), dt=0.005, max_steps=150, threshold=1e3),
    dict(n=32, A=4.0, sigma=(1.6, 1.3, 1.8), dt=0.005, max_steps=300, threshold=1e3),
    dict(n=48, A=0.6, sigma=(0.5, 0.6, 0.7), dt=0.005, max_steps=90, threshold=1e3),
    # the sweep's large classes (most of its kernel time): one blow-up and one
    # finished run each
    dict(n=96, A=3.0, sigma=(1.2, 0.9, 1.5), dt=0.005, max_steps=400, threshold=1e3),
    dict(n=96, A=1.0, sigma=(0.8, 1.3, 1.0), dt=0.005, max_steps=200, threshold=1e3),
    dict(n=128, A=3.5, sigma=(1.0, 1.4, 1.1), dt=0.005, max_steps=300, threshold=1e3),
    dict(n=128, A=1.4, sigma=(1.1, 0.7, 0.9), dt=0.005, max_steps=150, threshold=1e3),
]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_cases.json")


def single(kg, r):
    u0 = ki.gaussian(r["n"], r["A"], r["sigma"])
    with kg.Solver(r["n"], r["dt"], blowup_threshold=r["threshold"]) as s:
        s.set_state(u0)
        E0, _ = s.energy()
        st, done = s.step(r["max_steps"])
        steps, blown, bstep = s.stats()
        rec = s.records(0, bstep + 1 if blown else steps)
        E = s.energy()[0] if not blown else float("nan")
    return dict(blew_up=blown, steps_done=bstep if blown else steps, E0=E0, E_final=E,
                max_abs_u=float(np.nanmax(rec[2])))


def test_batch_matches_single_runs(kg):
    res, secs = kg.kg_batch_run(RUNS)
    assert secs > 0
    assert any(r["blew_up"] for r in res) and not all(r["blew_up"] for r in res)
    for r, b in zip(RUNS, res):
        s = single(kg, r)
        assert b["blew_up"] == s["blew_up"]
        assert b["steps_done"] == s["steps_done"]
        assert abs(b["E0"] - s["E0"]) <= 1e-11 * abs(s["E0"])
        if s["blew_up"]:
            assert abs(b["t_blowup"] - s["steps_done"] * r["dt"]) < 1e-12
            assert np.isnan(b["E_final"])
        else:
            assert b["t_blowup"] == -1.0
            assert abs(b["E_final"] - s["E_final"]) <= 1e-11 * abs(s["E_final"])
        assert abs(b["max_abs_u"] - s["max_abs_u"]) <= 1e-11 * s["max_abs_u"]


def test_batch_runs_are_independent(kg):
    """A poisoned run (it blows up at level 0) leaves the others bitwise unchanged."""
    base, _ = kg.kg_batch_run(RUNS)
    poison = dict(n=64, A=5e3, sigma=(1.0, 1.0, 1.0), dt=0.005, max_steps=100, threshold=1e3)
    mixed, _ = kg.kg_batch_run(RUNS[:2] + [poison] + RUNS[2:])
    assert mixed[2]["blew_up"] and mixed[2]["steps_done"] == 0
    for a, b in zip(base, mixed[:2] + mixed[3:]):
        for k in ("blew_up", "steps_done", "t_blowup", "max_abs_u"):
            assert a[k] == b[k]
        assert a["E0"] == b["E0"]
        assert (np.isnan(a["E_final"]) and np.isnan(b["E_final"])) or a["E_final"] == b["E_final"]


def test_batch_oracle_parity(kg):
    """Two 32^3 runs against the CPU oracle (blow-up step, E0, final energy)."""
    runs = [dict(n=32, A=1.2, sigma=(0.9, 1.1, 1.3), dt=0.01, max_steps=60, threshold=1e3),
            dict(n=32, A=4.0, sigma=(1.0, 1.2, 0.9), dt=0.01, max_steps=400, threshold=1e3)]
    res, _ = kg.kg_batch_run(runs)
    for r, b in zip(runs, res):
        ref = oracle.run(ki.gaussian(32, r["A"], r["sigma"]), r["dt"], r["max_steps"],
                         threshold=r["threshold"])
        assert b["blew_up"] == (ref["blowup_step"] >= 0)
        assert abs(b["E0"] - ref["energy"][0]) <= 1e-11 * abs(ref["energy"][0])
        if b["blew_up"]:
            assert b["steps_done"] == ref["blowup_step"]
        else:
            E = ref["energy"][r["max_steps"]]
            assert abs(b["E_final"] - E) <= 1e-11 * abs(E)


def test_batch_large_sizes_match_oracle(kg):
    """96^3 and 128^3 runs (radix-3 and power-of-two plans of the sweep's
    largest classes) against the oracle's runs (tests/golden/batch_cases.json,
    written by tests/golden/make_full_size.py from oracle/ only): blow-up
    level exact; E^{-1/2}, the final energy and max|u| to 1e-11 relative.
    For a blown run max|u| is taken at the blown level b, where the run
    amplifies perturbations: the reference file holds the oracle's response
    to data scaled by 1 + 1e-13, i.e. the amplification kappa of a relative
    perturbation.  The two sides differ by rounding of ~1e-15 per level,
    accumulating like a random walk over the b levels and amplified by at
    most kappa, so max|u| is held to 10 kappa 1e-15 sqrt(b) when that exceeds
    1e-11."""
    cases = json.load(open(GOLDEN))["cases"]
    runs = [dict(n=c["n"], A=c["A"], sigma=tuple(c["sigma"]), dt=c["dt"],
                 max_steps=c["max_steps"], threshold=c["threshold"]) for c in cases]
    res, _ = kg.kg_batch_run(runs)
    assert any(b["blew_up"] for b in res) and not all(b["blew_up"] for b in res)
    for c, b in zip(cases, res):
        ref, pert = c["ref"], c["perturbed_1e13"]
        assert b["blew_up"] == (ref["blowup_step"] >= 0)
        assert abs(b["E0"] - ref["E0"]) <= 1e-11 * abs(ref["E0"])
        kappa = abs(pert["max_abs_u"] - ref["max_abs_u"]) / ref["max_abs_u"] / 1e-13
        levels = ref["blowup_step"] if ref["blowup_step"] >= 0 else c["max_steps"]
        tol_max = max(1e-11, 10 * kappa * 1e-15 * np.sqrt(levels))
        assert abs(b["max_abs_u"] - ref["max_abs_u"]) <= tol_max * ref["max_abs_u"], (c, b)
        if b["blew_up"]:
            assert b["steps_done"] == ref["blowup_step"]
            assert abs(b["t_blowup"] - ref["blowup_step"] * c["dt"]) < 1e-12
        else:
            assert b["steps_done"] == c["max_steps"]
            assert abs(b["E_final"] - ref["E_final"]) <= 1e-11 * abs(ref["E_final"])


def test_batch_sweep_sizes_and_autotuner(kg, tmp_path):
    """The sweep's grid sizes, with the autotuner writing its cache: per size
    the tile width, the persistent workgroups per CU and the chunk size.  The
    tuned launches give the defaults' results: bitwise for the blow-up
    levels and max|u| (workgroups and chunks only change who computes a
    column, and a maximum has no order), energies to 1e-13 (a different tile
    width regroups the per-workgroup energy partials)."""
    runs = [dict(n=n, A=A, sigma=(1.0, 0.8, 1.2), dt=0.005, max_steps=40, threshold=1e3)
            for n in ki.SWEEP_SIZES for A in (0.7, 3.0)]
    cache = str(tmp_path / "tune.json")
    res, _ = kg.kg_batch_run(runs, tune=True, tune_cache=cache)
    table = json.load(open(cache))
    assert set(table) == {f"fp64/{n}/{k}" for n in ki.SWEEP_SIZES for k in ("W", "wpc", "chunk_mb")}
    for n in ki.SWEEP_SIZES:
        assert table[f"fp64/{n}/W"] in (4, 8)
        assert table[f"fp64/{n}/wpc"] in (2, 3, 4)
        assert table[f"fp64/{n}/chunk_mb"] in (200, 400, 800)
    ref, _ = kg.kg_batch_run(runs)  # defaults, no cache
    for a, b in zip(res, ref):
        for k in ("blew_up", "steps_done", "t_blowup", "max_abs_u"):
            assert a[k] == b[k], k
        assert abs(a["E0"] - b["E0"]) <= 1e-13 * abs(b["E0"])
        assert (np.isnan(a["E_final"]) and np.isnan(b["E_final"])) or \
            abs(a["E_final"] - b["E_final"]) <= 1e-13 * abs(b["E_final"])
    res2, _ = kg.kg_batch_run(runs, tune=True, tune_cache=cache)  # cached widths reused
    for a, b in zip(res, res2):
        assert a["blew_up"] == b["blew_up"] and a["steps_done"] == b["steps_done"]
        assert a["E0"] == b["E0"]
    for r, b in zip(runs, res):
        if r["A"] < 1:
            assert not b["blew_up"] and b["steps_done"] == 40


def test_batch_tests_every_level_like_the_oracle(kg):
    """The oracle tests every level 0..nsteps for blow-up, the last one too,
    and so must the sweep: a run whose blow-up level b equals max_steps is
    blown at b; with max_steps = b - 1 it finishes with the oracle's energy.
    Runs of zero steps report the initial pair's energy and max|u^0|, and one
    whose u0 already exceeds the threshold is blown at level 0, as is the same
    data given steps.  Close to a blow-up the run amplifies rounding, so the
    levels next to b are held to 1e-8 (E) and 1e-6 (max|u| above 1e3)
    instead of 1e-11."""
    dt, thr = 0.01, 1e3
    base = dict(n=32, A=4.0, sigma=(1.0, 1.2, 0.9), dt=dt, threshold=thr)
    u0 = ki.gaussian(32, base["A"], base["sigma"])
    ref = oracle.run(u0, dt, 400, threshold=thr)
    b = ref["blowup_step"]
    assert b > 2
    big = dict(base, A=2000.0)
    ref_big = oracle.run(ki.gaussian(32, big["A"], big["sigma"]), dt, 0, threshold=thr)
    assert ref_big["blowup_step"] == 0
    calm = dict(base, A=1.0, max_steps=20)
    ref_calm = oracle.run(ki.gaussian(32, calm["A"], calm["sigma"]), dt, 20, threshold=thr)
    runs = [dict(base, max_steps=b), dict(base, max_steps=b - 1), dict(base, max_steps=0),
            dict(big, max_steps=0), dict(big, max_steps=5), calm]
    res, _ = kg.kg_batch_run(runs)
    at_b, before_b, zero, big0, big5, calm_r = res
    rel = lambda x, y: abs(x - y) / abs(y)
    # blown exactly at its last level
    assert at_b["blew_up"] and at_b["steps_done"] == b and abs(at_b["t_blowup"] - b * dt) < 1e-12
    assert np.isnan(at_b["E_final"]) and at_b["max_abs_u"] > thr
    assert rel(at_b["max_abs_u"], np.max(ref["maxu"][:b + 1])) <= 1e-6
    # one step fewer: finished, with the oracle's energy of that level
    assert not before_b["blew_up"] and before_b["steps_done"] == b - 1
    assert rel(before_b["E_final"], ref["energy"][b - 1]) <= 1e-8
    assert rel(before_b["max_abs_u"], np.max(ref["maxu"][:b])) <= 1e-8
    # zero steps: level 0 only
    assert not zero["blew_up"] and zero["steps_done"] == 0 and zero["t_blowup"] == -1.0
    assert rel(zero["E0"], ref["energy"][0]) <= 1e-11 and zero["E_final"] == zero["E0"]
    assert rel(zero["max_abs_u"], ref["maxu"][0]) <= 1e-11
    for r in (at_b, before_b):
        assert rel(r["E0"], ref["energy"][0]) <= 1e-11
    # u0 above the threshold: blown at level 0 with or without steps
    for r in (big0, big5):
        assert r["blew_up"] and r["steps_done"] == 0 and r["t_blowup"] == 0.0
        assert np.isnan(r["E_final"])
        assert rel(r["E0"], ref_big["energy"][0]) <= 1e-11
        assert rel(r["max_abs_u"], ref_big["maxu"][0]) <= 1e-11
    # an ordinary run in the same batch is unaffected
    assert not calm_r["blew_up"] and calm_r["steps_done"] == 20
    assert rel(calm_r["E_final"], ref_calm["energy"][20]) <= 1e-11


def test_batch_rejects_an_empty_batch(kg):
    with pytest.raises(kg.KGError) as e:
        kg.kg_batch_run([])
    assert e.value.status == kg.KG_E_INVALID


def test_batch_rejects_bad_descriptors(kg):
    with pytest.raises(kg.KGError) as e:
        kg.kg_batch_run([dict(n=40, A=1, sigma=(1, 1, 1), dt=0.01, max_steps=5, threshold=0)])
    assert e.value.status == kg.KG_E_UNSUPPORTED_SIZE
    with pytest.raises(kg.KGError) as e:
        kg.kg_batch_run([dict(n=32, A=1, sigma=(1, 0, 1), dt=0.01, max_steps=5, threshold=0)])
    assert e.value.status == kg.KG_E_INVALID


def test_chunks_do_not_change_results(kg, monkeypatch):
    """Each size class steps chunk by chunk (a graph replays all its steps on
    one chunk before the next); runs are independent, so whole classes, the
    default chunks and one run per chunk give bitwise the same results."""
    runs = [dict(n=n, A=A, sigma=(1.0, 0.9, 1.2), dt=0.005, max_steps=300, threshold=1e3)
            for n in (32, 48) for A in (0.6, 1.4, 3.5, 5.0, 6.5)]
    out = {}
    for mb in ("0", None, "1"):  # 1 MB: every run is a chunk of its own
        if mb is None:
            monkeypatch.delenv("KG_BATCH_CHUNK_MB", raising=False)
        else:
            monkeypatch.setenv("KG_BATCH_CHUNK_MB", mb)
        out[mb], _ = kg.kg_batch_run(runs)
    assert any(r["blew_up"] for r in out["0"]) and not all(r["blew_up"] for r in out["0"])
    for mb in (None, "1"):
        for a, b in zip(out["0"], out[mb]):
            for k in ("blew_up", "steps_done", "t_blowup", "E0", "max_abs_u"):
                assert a[k] == b[k], (mb, k)
            assert (np.isnan(a["E_final"]) and np.isnan(b["E_final"])) or a["E_final"] == b["E_final"]
