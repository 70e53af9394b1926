"""The script that writes the full-size oracle references
(tests/golden/make_full_size.py) runs beyond 100 steps in segments joined by
two-level restarts from the physical pair (u^{m-1}, u^m).  A restart
re-transforms that pair, so it perturbs the run at the rounding level; this
checks that the segmented run stays within 1e-12 of one straight oracle run
(fields, energies, max|u| and Q4 at every level), far inside the 1e-11 the
GPU parity tests hold against the stored values.  CPU only; the case is a
nonlinear 32^3 Gaussian over 300 steps (three segments).
"""
import importlib.util
import os

import numpy as np

import kg_inputs as ki
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def load_script():
    spec = importlib.util.spec_from_file_location(
        "make_full_size", os.path.join(HERE, "golden", "make_full_size.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_segmented_reference_run_matches_a_straight_run(tmp_path, monkeypatch):
    mod = load_script()
    monkeypatch.setattr(mod, "HERE", str(tmp_path))
    n, A, sigma, levels = 32, 1.5, (1.0, 0.9, 1.1), (100, 300)
    mod.make_field(n, A, sigma, levels)
    g = np.load(os.path.join(tmp_path, mod.field_name(n, A)))
    ref = oracle.run(ki.gaussian(n, A, sigma), mod.DT, max(levels), threshold=mod.THRESHOLD)
    assert ref["blowup_step"] < 0
    for key in ("energy", "maxu", "q4"):
        a, b = g[key], ref[key]
        assert a.shape == b.shape
        assert np.max(np.abs(a - b) / np.abs(b)) <= 1e-12, key
    u = ref["u"]
    sub, blk, nrm = mod.samples(u)
    m = max(levels)
    assert np.linalg.norm(g[f"u{m}_sub"] - sub) <= 1e-12 * np.linalg.norm(sub)
    assert np.linalg.norm(g[f"u{m}_center"] - blk) <= 1e-12 * np.linalg.norm(blk)
    assert abs(g[f"u{m}_norm"] - nrm) <= 1e-12 * nrm
    # the first segment is the straight run itself
    r100 = oracle.run(ki.gaussian(n, A, sigma), mod.DT, 100, threshold=mod.THRESHOLD)
    assert np.array_equal(g["u100_sub"], mod.samples(r100["u"])[0])
