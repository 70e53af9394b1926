"""Pins of the oracle's optional dealiasing: the 2/3 rule applied to the
nonlinear term (an addition to the paper's plain pseudo-spectral scheme,
which has none; Sec. 1.1.2 forms the cubic term in physical space without
truncation).  A mode is kept when |m| <= n // 3 on every axis.

* After one step from two given levels, the dealiased and the plain v^1
  differ exactly on the removed modes, by beta_k F[u0^3]_k computed with
  numpy's FFT; the set of removed modes is checked against the rule on an
  anisotropic grid (cut-offs 8, 5 and 4).
* Band-limited data keeps a zero spectrum outside the kept box for all
  time: the removed modes evolve under the linear part only.
* A complex plane wave outside the box advances with the linear frequency
  cos(theta) = alpha / 2; inside it, with the nonlinear one.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle
from tests.test_oracle_complex import coeffs, wave

L = ki.BOX


def kept_box(shape):
    nz, ny, nx = shape
    mz, my, mx = (np.fft.fftfreq(n, 1.0 / n) for n in (nz, ny, nx))
    return ((np.abs(mz)[:, None, None] <= nz // 3) & (np.abs(my)[None, :, None] <= ny // 3) &
            (np.abs(mx)[None, None, :] <= nx // 3))


def betas(shape, Ls, dt):
    nz, ny, nx = shape
    kz, ky, kx = (2 * np.pi * np.fft.fftfreq(n, 1.0 / n) / Lx for n, Lx in zip((nz, ny, nx),
                                                                                 Ls[::-1]))
    w2 = 1 + kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    return dt * dt / (1 + w2 * dt * dt / 4)


def test_one_step_differs_exactly_on_the_removed_modes():
    shape, Ls, dt = (12, 16, 24), (L, 0.8 * L, 0.6 * L), 0.02   # (nz, ny, nx); L = (Lx, Ly, Lz)
    rng = np.random.default_rng(3)
    u0 = 0.8 * rng.standard_normal(shape)
    um1 = u0 + 0.01 * rng.standard_normal(shape)
    _, plain = oracle.state(u0, dt, 1, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1)
    _, dal = oracle.state(u0, dt, 1, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1, dealias=True)
    keep = kept_box(shape)
    assert keep.sum() == 9 * 11 * 17 and (~keep).sum() > 0
    assert np.array_equal(plain[keep], dal[keep])
    expected = betas(shape, Ls, dt) * np.fft.fftn(u0 ** 3)
    diff = plain - dal
    assert np.abs(diff[~keep] - expected[~keep]).max() <= 1e-12 * np.abs(expected).max()


def test_band_limited_data_stays_in_the_kept_box():
    n, dt, steps = 24, 0.01, 60
    rng = np.random.default_rng(7)
    spec = np.fft.fftn(rng.standard_normal((n, n, n)))
    spec[~kept_box((n, n, n))] = 0.0
    u0 = np.real(np.fft.ifftn(spec))
    u0 *= 1.5 / np.abs(u0).max()
    keep = kept_box((n, n, n))
    _, v = oracle.state(u0, dt, steps, dealias=True)
    assert np.abs(v[~keep]).max() <= 1e-12 * np.abs(v).max()
    _, v_plain = oracle.state(u0, dt, steps)
    assert np.abs(v_plain[~keep]).max() > 1e-6 * np.abs(v_plain).max()
    # the kept modes see the same scheme: closer to the plain run than the removed ones
    assert np.abs(v[keep] - v_plain[keep]).max() < np.abs(v_plain[~keep]).max()


@pytest.mark.parametrize("mode, inside", [((1, 2, -3), True), ((9, 0, 1), False),
                                          ((0, -6, 9), False), ((8, -8, 8), True)])
def test_plane_wave_frequency_follows_the_box(mode, inside):
    n, dt, steps, amp = 24, 0.01, 80, 0.8
    al, be = coeffs(n, dt, mode)
    th = np.arccos((al + (be * amp * amp if inside else 0.0)) / 2)
    r = oracle.run_complex(wave(n, mode, 0.0, amp), dt, steps, mode=oracle.INIT_TWO_LEVEL,
                           aux=wave(n, mode, th, amp), dealias=True)
    assert np.abs(r["u"] - wave(n, mode, -steps * th, amp)).max() <= 1e-11


def test_linear_runs_ignore_the_flag():
    n, dt = 16, 0.02
    u0 = ki.gaussian(n, 1.0, (0.9, 1.1, 1.2))
    a = oracle.run(u0, dt, 30, linear_only=True)
    b = oracle.run(u0, dt, 30, linear_only=True, dealias=True)
    assert np.array_equal(a["u"], b["u"])
