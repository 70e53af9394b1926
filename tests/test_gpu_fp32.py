"""FP32 path: FP32 FFTs and cubic term, FP64 update arithmetic and energy
reductions, time levels stored in increment form (v^n, v^n - v^{n-1}).

The stated target is a relative L2 error of at most 1e-4 against the FP64
solution.  Transform tolerances follow from FP32 rounding: a length-n FFT
accumulates about log2(n) roundings of 6e-8 relative to the largest
magnitude, plus a few ulp from derived twiddles, so 1e-5 of the maximum
bounds it with margin.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle

pytestmark = pytest.mark.gpu

FP32 = 1


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [8, 16, 24, 48, 64, 96, 256])
def test_fp32_transforms(kg, n):
    with kg.Solver(n, 0.01, precision=FP32) as s:
        u = ki.random_field(n, seed=n)
        got = kg.kg_debug_forward(s.plan, u)
        ref = oracle.fft3d(u)[:, :, :n // 2 + 1]
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
        back = kg.kg_debug_inverse(s.plan, ref)
        assert np.abs(back - u * n ** 3).max() <= 1e-5 * np.abs(u * n ** 3).max()


def test_fp32_small_config(kg):
    n, dt, steps = 32, 0.01, 100
    u0 = ki.gaussian(n, 0.1)
    ref = oracle.run(u0, dt, steps)
    with kg.Solver(n, dt, precision=FP32) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
    assert rel_l2(u, ref["u"]) <= 1e-4
    assert abs(E - ref["energy"][steps]) <= 1e-4 * abs(ref["energy"][steps])


@pytest.mark.parametrize("n, sigma", [(128, (1.0, 1.0, 1.0)), (48, (0.8, 1.1, 1.3)), (96, (1.3, 0.9, 1.0))])
def test_fp32_nonlinear_against_oracle(kg, n, sigma):
    """A = 1.5 Gaussian (the precision study's data) at 128^3, and the
    3 * 2^a grids of the sweep (radix-3 lines, 12 values per thread) with
    anisotropic widths, 200 steps."""
    dt, steps = 0.005, 200
    u0 = ki.gaussian(n, 1.5, sigma)
    ref = oracle.run(u0, dt, steps)
    with kg.Solver(n, dt, precision=FP32) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
        elin, q4, _ = s.records(0, steps)
        E, _ = s.energy()
    err = rel_l2(u, ref["u"])
    assert err <= 1e-4, err
    assert abs(E - ref["energy"][steps]) <= 1e-4 * abs(ref["energy"][steps])


def test_fp32_plane_wave(kg):
    n, dt, steps, mode = 32, 0.01, 100, (4, 8, 0)
    k = 2 * np.pi * np.asarray(mode) / ki.BOX
    w = np.sqrt(1 + (k * k).sum())
    th = 2 * np.arctan(w * dt / 2)
    with kg.Solver(n, dt, linear_only=True, precision=FP32) as s:
        s.set_state(ki.plane_wave(n, mode), ki.plane_wave(n, mode, th), kg.KG_INIT_TWO_LEVEL)
        s.step(steps)
        u = s.u()
    assert rel_l2(u, ki.plane_wave(n, mode, -steps * th)) <= 1e-5


def test_fp32_blowup_step(kg):
    """Uniform a = 1.5 blows up at step 145 in FP64; FP32 storage may move
    the threshold crossing by at most one step."""
    with kg.Solver(8, 0.01, blowup_threshold=1e3, precision=FP32) as s:
        s.set_state(ki.uniform(8, 1.5))
        st, _ = s.step(300)
        _, blown, bstep = s.stats()
    assert st == kg.KG_BLOWUP and blown and abs(bstep - 145) <= 1


def test_fp32_determinism_and_checkpoint(kg):
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.5, (0.9, 1.1, 1.3))
    with kg.Solver(n, dt, precision=FP32) as a, kg.Solver(n, dt, precision=FP32) as b:
        a.set_state(u0)
        b.set_state(u0)
        a.step(60)
        b.step(30)
        blob = b.save()
        b.set_state(ki.gaussian(n, 0.2))
        b.load(blob)
        b.step(30)
        assert np.array_equal(a.u(), b.u())
        assert a.energy() == b.energy()
        assert np.array_equal(a.spectrum(1), b.spectrum(1))
