"""Planted mistakes in the oracle (on the CPU, in a copy of its source) must
each be caught by at least one of the pins.  This is evidence that the pins
constrain every part of the oracle: transform, wavenumbers, scheme
coefficients, start-up rule, cubic term and energy.
"""
import os

import numpy as np
import pytest

import kg_inputs as ki
import oracle
from oracle.build import SRC, build_oracle
from tests.test_oracle_complex import charge, coeffs, wave
from tests.test_oracle_dealias import betas, kept_box
from tests.test_oracle_pins import (cd_solution, dense_laplacian, gaussian_energy,
                                    omega_of_mode)

L = ki.BOX

MUTANTS = {
    "twiddle_sign": ("tw[j] = cos(ang) + (double)sign * sin(ang) * I;",
                     "tw[j] = cos(ang) + sin(ang) * I;"),
    "combine_index": ("out[k1 + (ptrdiff_t)s * m] = acc;", "out[(ptrdiff_t)k1 * p + s] = acc;"),
    "twiddle_skip": ("y[r] = out[(ptrdiff_t)r * m + k1] * tw[(r * k1 * ts) % N];",
                     "y[r] = out[(ptrdiff_t)r * m + k1];"),
    "wavenumber_no_wrap": ("return i <= n / 2 ? i : i - n;", "return i;"),
    "axis_box_swap": ("double ky = 2.0 * M_PI * mode_number(iy, g->ny) / g->Ly;",
                      "double ky = 2.0 * M_PI * mode_number(iy, g->ny) / g->Lx;"),
    "alpha_sign": ("*alpha = 2.0 * (1.0 - a) / (1.0 + a);", "*alpha = 2.0 * (1.0 + a) / (1.0 + a);"),
    "beta_no_denominator": ("*beta = g->dt * g->dt / (1.0 + a);", "*beta = g->dt * g->dt;"),
    "a_factor": ("double a = omega2(g, ix, iy, iz) * g->dt * g->dt / 4.0;",
                 "double a = omega2(g, ix, iy, iz) * g->dt * g->dt / 2.0;"),
    "mass_term_dropped": ("return 1.0 + kx * kx + ky * ky + kz * kz;",
                          "return kx * kx + ky * ky + kz * kz;"),
    "start_velocity_sign": ("vp[i] = 0.5 * al * vc[i] - g->dt * vp[i] + 0.5 * be * w[i];",
                            "vp[i] = 0.5 * al * vc[i] + g->dt * vp[i] + 0.5 * be * w[i];"),
    "start_cubic_dropped": ("vp[i] = 0.5 * al * vc[i] - g->dt * vp[i] + 0.5 * be * w[i];",
                            "vp[i] = 0.5 * al * vc[i] - g->dt * vp[i];"),
    "square_not_cube": ("cube[i] = g->chi * cube[i] * cube[i] * cube[i];",
                        "cube[i] = g->chi * cube[i] * cube[i];"),
    "cubic_sign": ("vp[i] = al * vc[i] - vp[i] + be * w[i];", "vp[i] = al * vc[i] - vp[i] - be * w[i];"),
    "inverse_not_normalised": ("double x = creal(work[i]) / (double)M;", "double x = creal(work[i]);"),
    "energy_quartic_weight": ("energy[n] = elin_prev - g.chi * (q4_prev + st.q4) / 8.0;",
                              "energy[n] = elin_prev - g.chi * (q4_prev + st.q4) / 4.0;"),
    "energy_kinetic_dt": ("s += dd / (g->dt * g->dt) + w2 * pp / 4.0;", "s += dd / g->dt + w2 * pp / 4.0;"),
    "energy_level_mix": ("elin_prev = linear_energy(&g, vc, vp);", "elin_prev = linear_energy(&g, vc, vc);"),
    # complex fields
    "complex_u_cubed": ("tmp[i] = g->chi * m2 * u[i];", "tmp[i] = g->chi * u[i] * u[i] * u[i];"),
    "complex_modulus_real_part": (
        "double m2 = creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);",
        "double m2 = creal(u[i]) * creal(u[i]);"),
    "complex_imag_dropped": ("cplx x = u[i] / (double)M;", "cplx x = creal(u[i]) / (double)M;"),
    "complex_inverse_sign": ("fft3d_axis(g->nx, g->ny, g->nz, u, 0, 1)",
                             "fft3d_axis(g->nx, g->ny, g->nz, u, 0, -1)"),
    "complex_quartic_real_part": ("s4 += m2 * m2;",
                                  "s4 += creal(x) * creal(x) * creal(x) * creal(x);"),
    # dealiasing
    "dealias_cutoff_strict": ("abs(mode_number(ix, g->nx)) <= g->nx / 3",
                              "abs(mode_number(ix, g->nx)) < g->nx / 3"),
    "dealias_axis_mix": ("abs(mode_number(iy, g->ny)) <= g->ny / 3",
                         "abs(mode_number(iy, g->ny)) <= g->nx / 3"),
    "dealias_skipped_in_steps": (
        "cube[i] = g->chi * cube[i] * cube[i] * cube[i];\n    if (forward_real(g, cube, w))\n"
        "        return KGO_ENOMEM;\n    truncate_nonlinear(g, w);",
        "cube[i] = g->chi * cube[i] * cube[i] * cube[i];\n    if (forward_real(g, cube, w))\n"
        "        return KGO_ENOMEM;"),
    "dealias_skipped_complex": ("    if (forward_cplx(g, tmp, w))\n        return KGO_ENOMEM;\n"
                                "    truncate_nonlinear(g, w);",
                                "    if (forward_cplx(g, tmp, w))\n        return KGO_ENOMEM;"),
}


def battery(o):
    """The pins in compact form; returns the names of those that fail."""
    failed = []
    rng = np.random.default_rng(5)
    # transform vs the DFT definition
    for n in (12, 16):
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        j = np.arange(n)
        ref = np.exp(-2j * np.pi * (np.outer(j, j) % n) / n) @ x
        if np.abs(o.fft1d(x) - ref).max() > 1e-12 * np.abs(ref).max():
            failed.append("fft1d")
    # discrete plane wave, anisotropic grid and box
    Ls = (L, 0.75 * L, 0.5 * L)
    mode = (3, -5, 2)
    dt = 0.01
    w = omega_of_mode(mode, Ls)
    th = 2 * np.arctan(w * dt / 2)
    r = o.run(ki.plane_wave((16, 24, 12), mode, 0.0, Ls), dt, 30, L=Ls, linear_only=True,
              mode=oracle.INIT_TWO_LEVEL, aux=ki.plane_wave((16, 24, 12), mode, th, Ls))
    ex = ki.plane_wave((16, 24, 12), mode, -30 * th, Ls)
    if not np.linalg.norm(r["u"] - ex) <= 1e-11 * np.linalg.norm(ex):
        failed.append("plane_wave")
    # velocity start closed form
    mode = (4, 8, 0)
    w = omega_of_mode(mode)
    dt = 0.05
    th = 2 * np.arctan(w * dt / 2)
    a = w * w * dt * dt / 4
    r = o.run(ki.plane_wave(16, mode), dt, 9, linear_only=True,
              aux=w * ki.plane_wave(16, mode, fn=np.sin))
    ex = ki.plane_wave(16, mode, -9 * th) + a * np.sin(9 * th) * ki.plane_wave(16, mode, fn=np.sin)
    if not np.abs(r["u"] - ex).max() <= 1e-11:
        failed.append("velocity_start")
    # eq. (2) as a dense solve
    nx, ny, nz = 6, 4, 8
    Ls = (L, 0.6 * L, 1.3 * L)
    dt = 0.05
    um1 = 0.8 * ki.gaussian((nx, ny, nz), 1.0, (5.0, 3.0, 6.0), Ls) + \
        0.1 * rng.standard_normal((nz, ny, nx))
    u0 = um1 + 0.05 * rng.standard_normal((nz, ny, nx))
    lap = dense_laplacian(nx, ny, nz, Ls)
    I = np.eye(nx * ny * nz)
    A = I / dt ** 2 + (I - lap) / 4
    up, uc = um1.ravel(), u0.ravel()
    for _ in range(3):
        rhs = uc ** 3 + (2 * uc - up) / dt ** 2 - (I - lap) @ (2 * uc + up) / 4
        up, uc = uc, np.linalg.solve(A, rhs)
    r = o.run(u0, dt, 3, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1)
    if not np.abs(r["u"].ravel() - uc).max() <= 1e-11 * np.abs(uc).max():
        failed.append("dense_eq2")
    # uniform data vs the ODE's closed form, second order
    errs = []
    for dt in (0.02, 0.01):
        rr = o.run(ki.uniform(4, 0.5), dt, int(round(4 / dt)))
        errs.append(abs(rr["u"][0, 0, 0] - cd_solution(0.5, 4.0)))
    if not (errs[0] < 1e-4 and 3.5 < errs[0] / errs[1] < 4.5):
        failed.append("uniform_ode")
    # energy: closed form at the start, exact linear conservation, O(dt^2) drift
    rr = o.run(ki.gaussian(64, 1.5), 1e-4, 0)
    if not abs(rr["energy"][0] - gaussian_energy(1.5, (1, 1, 1))) < 1e-5:
        failed.append("energy_closed_form")
    rr = o.run(ki.gaussian(16, 0.5, (1.5, 1.7, 2.0)), 0.02, 20, linear_only=True)
    if not np.abs(rr["energy"] - rr["energy"][0]).max() <= 1e-12 * abs(rr["energy"][0]):
        failed.append("linear_energy")
    drifts = []
    for dt in (0.02, 0.01):
        rr = o.run(ki.gaussian(16, 1.5, (1.5, 1.7, 2.0)), dt, int(round(0.4 / dt)))
        drifts.append(np.abs(rr["energy"] - rr["energy"][0]).max() / abs(rr["energy"][0]))
    if not (drifts[0] < 1e-2 and 3.0 < drifts[0] / drifts[1] < 5.0):
        failed.append("nonlinear_energy")
    # complex field: nonlinear plane wave (|u|^2 u keeps it), its energy in
    # closed form, and the discrete charge
    n, dt, cm, amp = 16, 0.01, (1, 2, -3), 0.8
    al, be = coeffs(n, dt, cm)
    th = np.arccos((al + be * amp * amp) / 2)
    r = o.run_complex(wave(n, cm, 0.0, amp), dt, 40, mode=oracle.INIT_TWO_LEVEL,
                      aux=wave(n, cm, th, amp))
    if not np.abs(r["u"] - wave(n, cm, -40 * th, amp)).max() <= 1e-11:
        failed.append("complex_plane_wave")
    k = 2 * np.pi * np.asarray(cm, float) / L
    w2 = 1.0 + np.sum(k * k)
    e = L ** 3 * amp ** 2 / 2 * (4 * np.sin(th / 2) ** 2 / dt ** 2 + w2 * np.cos(th / 2) ** 2) \
        - L ** 3 * amp ** 4 / 4
    if not np.allclose(r["energy"], e, rtol=1e-12, atol=0):
        failed.append("complex_energy")
    z, y, x = ki.mesh(n, L)
    u0 = ki.gaussian(n, 1.1, (1.0, 0.8, 1.2)) * np.exp(1j * 0.6 * (x - 0.5 * y + 0.3 * z))
    r0 = o.run_complex(u0, dt, 0, aux=0.4j * u0)
    r1 = o.run_complex(u0, dt, 30, aux=0.4j * u0)
    c0, c1 = charge(n, dt, r0["u_prev"], r0["u"]), charge(n, dt, r1["u_prev"], r1["u"])
    if not (abs(c0) > 1.0 and abs(c1 - c0) <= 1e-12 * abs(c0)):
        failed.append("complex_charge")
    # dealiasing: one step differs from the plain one by beta F[u0^3] exactly
    # on the removed modes; band-limited data stays in the box; a complex
    # plane wave outside the box advances linearly
    shape, Ls, dt = (12, 16, 24), (L, 0.8 * L, 0.6 * L), 0.02
    u0 = 0.8 * rng.standard_normal(shape)
    um1 = u0 + 0.01 * rng.standard_normal(shape)
    _, plain = o.state(u0, dt, 1, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1)
    _, dal = o.state(u0, dt, 1, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1, dealias=True)
    keep = kept_box(shape)
    exp = betas(shape, Ls, dt) * np.fft.fftn(u0 ** 3)
    if not (np.array_equal(plain[keep], dal[keep]) and
            np.abs((plain - dal)[~keep] - exp[~keep]).max() <= 1e-12 * np.abs(exp).max()):
        failed.append("dealias_one_step")
    n = 24
    spec = np.fft.fftn(rng.standard_normal((n, n, n)))
    spec[~kept_box((n, n, n))] = 0.0
    ub = np.real(np.fft.ifftn(spec))
    ub *= 1.5 / np.abs(ub).max()
    _, v = o.state(ub, 0.01, 20, dealias=True)
    if not np.abs(v[~kept_box((n, n, n))]).max() <= 1e-12 * np.abs(v).max():
        failed.append("dealias_band_limited")
    cm, amp = (9, 0, 1), 0.8
    al, be = coeffs(n, 0.01, cm)
    th = np.arccos(al / 2)
    r = o.run_complex(wave(n, cm, 0.0, amp), 0.01, 40, mode=oracle.INIT_TWO_LEVEL,
                      aux=wave(n, cm, th, amp), dealias=True)
    if not np.abs(r["u"] - wave(n, cm, -40 * th, amp)).max() <= 1e-11:
        failed.append("dealias_complex_wave")
    return failed


def test_battery_passes_on_the_oracle():
    assert battery(oracle.default()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new, 1))
    lib = build_oracle(str(path), str(tmp_path / "libmutant.so"))
    o = oracle.Oracle(lib)
    failed = battery(o)
    assert failed, f"mutant {name} passed every pin"
