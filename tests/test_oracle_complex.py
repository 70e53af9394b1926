"""Pins of the oracle's complex-field path (the benchmark code of Sec. 1.1.2
also allows complex u; the cubic term is then |u|^2 u, Sec. 1):

* real data stepped as a complex field reproduces the real path;
* a plane wave is an exact discrete solution of eq. (2), in the linear case
  and, because |u|^2 stays constant, in the nonlinear one with the shifted
  frequency cos(theta) = (alpha + beta a^2) / 2 (a cubic u^3 would instead
  feed the third harmonic);
* the discrete charge C = sum_k (1 + a_k) Im(conj(v^n_k) v^{n+1}_k) is
  conserved exactly by eq. (2) with the |u|^2 u term (multiply eq. (2) by
  (1 + a_k) conj(v^n_k), take imaginary parts and sum: the nonlinear part is
  Im sum_j |u_j|^4 = 0 by Parseval), and the linear energy is conserved.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle

L = ki.BOX


def coeffs(n, dt, modes):
    k = 2 * np.pi * np.asarray(modes, float) / L
    w2 = 1.0 + np.sum(k * k)
    a = w2 * dt * dt / 4
    return 2 * (1 - a) / (1 + a), dt * dt / (1 + a)


def wave(n, mode, phase, amp=1.0):
    z, y, x = ki.mesh(n, L)
    k = 2 * np.pi * np.asarray(mode, float) / L
    return amp * np.exp(1j * (k[0] * x + k[1] * y + k[2] * z + phase))


def test_real_data_matches_the_real_path():
    u0 = ki.gaussian(16, 1.3, (0.9, 1.1, 1.3))
    a = oracle.run(u0, 0.01, 40)
    b = oracle.run_complex(u0.astype(complex), 0.01, 40)
    assert np.abs(b["u"].real - a["u"]).max() <= 1e-13 * np.abs(a["u"]).max()
    assert np.abs(b["u"].imag).max() <= 1e-13 * np.abs(a["u"]).max()
    assert np.allclose(b["energy"], a["energy"], rtol=1e-13, atol=0)
    assert np.allclose(b["maxu"], a["maxu"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("amp, linear", [(1.0, True), (0.7, False), (1.3, False)])
def test_plane_wave_is_exact(amp, linear):
    n, dt, steps, mode = 16, 0.01, 100, (1, 2, -3)
    al, be = coeffs(n, dt, mode)
    c = (al + (0.0 if linear else be * amp * amp)) / 2
    th = np.arccos(c)
    r = oracle.run_complex(wave(n, mode, 0.0, amp), dt, steps, linear_only=linear,
                           mode=oracle.INIT_TWO_LEVEL, aux=wave(n, mode, th, amp))
    exact = wave(n, mode, -steps * th, amp)
    assert np.abs(r["u"] - exact).max() <= 1e-11 * amp
    assert np.allclose(r["maxu"], amp, rtol=1e-12)


def test_cubic_u3_would_not_keep_the_plane_wave():
    """The pin above separates |u|^2 u from u^3: one step of u^3 from the
    same wave leaves the single mode."""
    n, mode = 16, (1, 2, -3)
    u = wave(n, mode, 0.0, 1.0)
    spec = np.abs(oracle.fft3d(u ** 3))
    spec_ok = np.abs(oracle.fft3d(np.abs(u) ** 2 * u))
    assert (spec > 1e-6 * spec.max()).sum() == 1 and (spec_ok > 1e-6 * spec_ok.max()).sum() == 1
    assert np.argmax(spec) != np.argmax(spec_ok)  # u^3 sits on mode 3k, |u|^2 u on k


def charge(n, dt, up, u):
    vp, v = oracle.fft3d(up), oracle.fft3d(u)
    m = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    w2 = 1 + (2 * np.pi / L) ** 2 * (kx * kx + ky * ky + kz * kz)
    return np.sum((1 + w2 * dt * dt / 4) * np.imag(np.conj(vp) * v))


def test_discrete_charge_and_linear_energy_are_conserved():
    n, dt = 16, 0.01
    z, y, x = ki.mesh(n, L)
    u0 = ki.gaussian(n, 1.1, (1.0, 0.8, 1.2)) * np.exp(1j * 0.6 * (x - 0.5 * y + 0.3 * z))
    ut0 = 0.4j * u0  # a rotating phase: nonzero charge
    r0 = oracle.run_complex(u0, dt, 0, aux=ut0)
    r1 = oracle.run_complex(u0, dt, 60, aux=ut0)
    c0, c1 = charge(n, dt, r0["u_prev"], r0["u"]), charge(n, dt, r1["u_prev"], r1["u"])
    assert abs(c0) > 1.0
    assert abs(c1 - c0) <= 1e-12 * abs(c0)
    rl = oracle.run_complex(u0, dt, 60, aux=ut0, linear_only=True)
    assert np.abs(rl["energy"] - rl["energy"][0]).max() <= 1e-12 * abs(rl["energy"][0])
    # with the nonlinear term the energy drifts at O(dt^2) only
    assert np.abs(r1["energy"] - r1["energy"][0]).max() <= 1e-3 * abs(r1["energy"][0])


@pytest.mark.parametrize("amp", [0.5, 0.9])
def test_plane_wave_energy_closed_form(amp):
    """For a plane wave of amplitude A advancing by theta per step, the
    discrete energy has the closed form
    (L^3 A^2 / 2) [4 sin^2(theta/2) / dt^2 + omega^2 cos^2(theta/2)] - L^3 A^4 / 4
    (the linear pair energy of Sec. 1.1 with a single mode, minus the
    quartic term at two equal levels)."""
    n, dt, steps, mode = 16, 0.01, 20, (2, -1, 1)
    al, be = coeffs(n, dt, mode)
    th = np.arccos((al + be * amp * amp) / 2)
    k = 2 * np.pi * np.asarray(mode, float) / L
    w2 = 1.0 + np.sum(k * k)
    e = L ** 3 * amp ** 2 / 2 * (4 * np.sin(th / 2) ** 2 / dt ** 2 + w2 * np.cos(th / 2) ** 2) \
        - L ** 3 * amp ** 4 / 4
    r = oracle.run_complex(wave(n, mode, 0.0, amp), dt, steps, mode=oracle.INIT_TWO_LEVEL,
                           aux=wave(n, mode, th, amp))
    assert np.allclose(r["energy"], e, rtol=1e-12, atol=0)
