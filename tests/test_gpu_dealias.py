"""Parity of the optional 2/3-rule dealiasing on the GPU (the nonlinear
term keeps the modes with |m| <= n // 3 on every axis; an addition to the
paper's plain pseudo-spectral scheme) with the oracle's dealiased runs, and
with the properties that pin the rule: one step changes only the removed
modes, band-limited data stays in the kept box, and a complex plane wave
outside the box advances with the linear frequency.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle
from tests.test_gpu_complex import phased_gaussian
from tests.test_oracle_complex import coeffs, wave
from tests.test_oracle_dealias import kept_box

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,A,steps", [(48, 2.0, 60), (32, 1.5, 100), (64, 1.8, 40)])
def test_real_field_matches_oracle(kg, n, A, steps):
    dt = 0.005
    u0 = ki.gaussian(n, A, (0.7, 1.0, 1.2)) + ki.gaussian(n, 0.3, (1.0, 1.0, 1.0),
                                                            center=(2.0, -1.0, 0.5))
    ref = oracle.run(u0, dt, steps, dealias=True)
    plain = oracle.run(u0, dt, steps)
    assert rel_l2(plain["u"], ref["u"]) > 1e-9  # the truncation matters for this data
    with kg.Solver(n, dt, dealias=True) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
        _, q4, maxu = s.records(0, steps)
    assert rel_l2(u, ref["u"]) <= 1e-11
    assert abs(E - ref["energy"][steps]) <= 1e-11 * abs(ref["energy"][steps])
    assert np.allclose(maxu, ref["maxu"][:steps], rtol=1e-11, atol=0)


@pytest.mark.parametrize("precision,tol", [(0, 1e-11), (1, 1e-4)])
def test_complex_field_matches_oracle(kg, precision, tol):
    n, dt, steps = 48, 0.005, 60
    u0 = phased_gaussian(n, 1.8, (0.7, 1.2, 0.9), (0.0, 0.8, -0.5))
    ref = oracle.run_complex(u0, dt, steps, aux=0.3j * u0, dealias=True)
    with kg.Solver(n, dt, precision=precision, complex_field=True, dealias=True) as s:
        s.set_state(u0, 0.3j * u0)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
    assert rel_l2(u, ref["u"]) <= tol
    assert abs(E - ref["energy"][steps]) <= tol * abs(ref["energy"][steps])


def test_fp32_real_field_matches_oracle(kg):
    n, dt, steps = 96, 0.005, 40
    u0 = ki.gaussian(n, 1.5, (0.6, 0.9, 1.2))
    ref = oracle.run(u0, dt, steps, dealias=True)
    with kg.Solver(n, dt, precision=kg.KG_FP32, dealias=True) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
    assert rel_l2(u, ref["u"]) <= 1e-4


def test_one_step_changes_only_the_removed_modes(kg):
    n, dt = 48, 0.01
    rng = np.random.default_rng(11)
    u0 = 0.8 * rng.standard_normal((n, n, n))
    um1 = u0 + 0.01 * rng.standard_normal((n, n, n))
    spec = []
    for dealias in (False, True):
        with kg.Solver(n, dt, dealias=dealias) as s:
            s.set_state(u0, um1, kg.KG_INIT_TWO_LEVEL)
            s.step(1)
            spec.append(s.spectrum(0))
    keep = kept_box((n, n, n))[:, :, :n // 2 + 1]
    assert np.array_equal(spec[0][keep], spec[1][keep])
    assert np.abs(spec[0][~keep] - spec[1][~keep]).min() > 0


def test_band_limited_data_stays_in_the_box(kg):
    n, dt, steps = 48, 0.01, 200
    rng = np.random.default_rng(7)
    full = np.fft.fftn(rng.standard_normal((n, n, n)))
    full[~kept_box((n, n, n))] = 0.0
    u0 = np.ascontiguousarray(np.real(np.fft.ifftn(full)))
    u0 *= 1.5 / np.abs(u0).max()
    keep = kept_box((n, n, n))[:, :, :n // 2 + 1]
    with kg.Solver(n, dt, dealias=True) as s:
        s.set_state(u0)
        s.step(steps)
        v = s.spectrum(0)
    assert np.abs(v[~keep]).max() <= 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("mode, inside", [((3, -5, 2), True), ((0, 12, -1), False),
                                          ((11, 11, 0), False), ((10, -10, 10), True)])
def test_complex_plane_wave_frequency_follows_the_box(kg, mode, inside):
    n, dt, steps, amp = 32, 0.01, 100, 0.8
    al, be = coeffs(n, dt, mode)
    th = np.arccos((al + (be * amp * amp if inside else 0.0)) / 2)
    with kg.Solver(n, dt, complex_field=True, dealias=True) as s:
        s.set_state(wave(n, mode, 0.0, amp), wave(n, mode, th, amp), kg.KG_INIT_TWO_LEVEL)
        s.step(steps)
        u = s.u()
    assert np.abs(u - wave(n, mode, -steps * th, amp)).max() <= 1e-11
