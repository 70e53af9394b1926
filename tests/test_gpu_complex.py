"""Parity of the complex-field path (u complex, cubic term |u|^2 u: Sec. 1;
the benchmark code of Sec. 1.1.2 also steps complex fields) with the
oracle's complex path and with the closed forms that pin it:

* the 3D transform of a complex field against numpy's FFT;
* real data stepped as a complex field reproduces the real path;
* a nonlinear plane wave is an exact discrete solution of eq. (2), with the
  energy in closed form;
* the discrete charge sum_k (1 + a_k) Im(conj(v^{n-1}_k) v^n_k) is conserved
  exactly by eq. (2) with |u|^2 u;
* Gaussians with a phase gradient match the oracle step by step, on grids
  of several tiles with ragged edges, in FP64 (1e-11) and FP32 (1e-4).
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle
from tests.test_oracle_complex import coeffs, wave

pytestmark = pytest.mark.gpu

L = ki.BOX


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def phased_gaussian(n, A, sigma, kvec, center=(0.0, 0.0, 0.0)):
    z, y, x = ki.mesh(n, L)
    return ki.gaussian(n, A, sigma, center=center) * np.exp(
        1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))


def spectral_charge(n, dt, vp, vc):
    """sum_k (1 + a_k) Im(conj(vp_k) vc_k) over the full spectrum."""
    m = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    w2 = 1 + (2 * np.pi / L) ** 2 * (kx * kx + ky * ky + kz * kz)
    return np.sum((1 + w2 * dt * dt / 4) * np.imag(np.conj(vp) * vc))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [8, 24, 48, 64])
def test_complex_transform_matches_numpy(kg, n, precision):
    rng = np.random.default_rng(n)
    u = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    ref = np.fft.fftn(u)
    tol = 1e-12 if precision == 0 else 1e-5
    with kg.Solver(n, 0.01, precision=precision, complex_field=True) as s:
        got = kg.kg_debug_forward(s.plan, u)
        back = kg.kg_debug_inverse(s.plan, ref)
    assert got.shape == (n, n, n)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    assert np.abs(back - u * n ** 3).max() <= tol * np.abs(u * n ** 3).max()


@pytest.mark.parametrize("precision", [0, 1])
def test_real_data_as_complex_field_matches_real_path(kg, precision):
    n, dt, steps = 48, 0.005, 40
    u0 = ki.gaussian(n, 1.6, (0.8, 1.1, 1.3))
    ut0 = ki.gaussian(n, 0.4, (1.0, 0.9, 1.2), center=(0.5, -1.0, 0.0))
    with kg.Solver(n, dt, precision=precision) as s:
        s.set_state(u0, ut0)
        s.step(steps)
        ur = s.u()
        Er, _ = s.energy()
        _, q4r, mxr = s.records(0, steps)
    with kg.Solver(n, dt, precision=precision, complex_field=True) as s:
        s.set_state(u0.astype(complex), ut0.astype(complex))
        s.step(steps)
        uc = s.u()
        Ec, _ = s.energy()
        _, q4c, mxc = s.records(0, steps)
    tol = 1e-12 if precision == 0 else 1e-5
    assert rel_l2(uc.real, ur) <= tol
    assert np.abs(uc.imag).max() <= tol * np.abs(ur).max()
    assert abs(Ec - Er) <= tol * abs(Er)
    assert np.allclose(q4c, q4r, rtol=10 * tol, atol=0)
    assert np.allclose(mxc, mxr, rtol=10 * tol, atol=0)


@pytest.mark.parametrize("amp", [0.5, 0.9])
def test_nonlinear_plane_wave_is_exact(kg, amp):
    """|u| stays constant, so |u|^2 u is a multiple of the single mode and
    the wave advances by theta per step, cos(theta) = (alpha + beta A^2) / 2;
    the energy is then
    (L^3 A^2 / 2) [4 sin^2(theta/2) / dt^2 + omega^2 cos^2(theta/2)] - L^3 A^4 / 4."""
    n, dt, steps, mode = 32, 0.01, 100, (3, -2, 5)
    al, be = coeffs(n, dt, mode)
    th = np.arccos((al + be * amp * amp) / 2)
    with kg.Solver(n, dt, complex_field=True) as s:
        s.set_state(wave(n, mode, 0.0, amp), wave(n, mode, th, amp), kg.KG_INIT_TWO_LEVEL)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
        _, _, maxu = s.records(0, steps)
    assert np.abs(u - wave(n, mode, -steps * th, amp)).max() <= 1e-11 * amp
    k = 2 * np.pi * np.asarray(mode, float) / L
    w2 = 1.0 + np.sum(k * k)
    e = L ** 3 * amp ** 2 / 2 * (4 * np.sin(th / 2) ** 2 / dt ** 2 + w2 * np.cos(th / 2) ** 2) \
        - L ** 3 * amp ** 4 / 4
    assert abs(E - e) <= 1e-11 * abs(e)
    assert np.allclose(maxu, amp, rtol=1e-12)


@pytest.mark.parametrize("n,A,sigma,kvec,steps", [(32, 1.2, (1.0, 0.8, 1.2), (0.6, -0.3, 0.2), 80),
                                                   (48, 1.8, (0.7, 1.2, 0.9), (0.0, 0.8, -0.5), 60),
                                                   (24, 1.0, (1.1, 1.0, 0.9), (1.0, 0.0, 0.0), 100),
                                                   (64, 1.5, (0.8, 1.0, 1.3), (-0.4, 0.5, 0.7), 40)])
def test_phased_gaussian_matches_oracle(kg, n, A, sigma, kvec, steps):
    dt = 0.005
    u0 = phased_gaussian(n, A, sigma, kvec) + phased_gaussian(n, 0.3, (1.0, 1.0, 1.0), (0.2, 0.1, 0),
                                                               center=(2.0, -1.0, 0.5))
    ut0 = 0.3j * u0
    ref = oracle.run_complex(u0, dt, steps, aux=ut0)
    with kg.Solver(n, dt, complex_field=True) as s:
        s.set_state(u0, ut0)
        E0, _ = s.energy()
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        u = s.u()
        E, _ = s.energy()
        elin, q4, maxu = s.records(0, steps)
    assert rel_l2(u, ref["u"]) <= 1e-11
    assert abs(E0 - ref["energy"][0]) <= 1e-11 * abs(ref["energy"][0])
    assert abs(E - ref["energy"][steps]) <= 1e-11 * abs(ref["energy"][steps])
    assert np.allclose(maxu, ref["maxu"][:steps], rtol=1e-11, atol=0)
    assert np.allclose(q4, ref["q4"][:steps], rtol=1e-10, atol=0)


@pytest.mark.parametrize("n", [32, 48])
def test_phased_gaussian_fp32(kg, n):
    dt, steps = 0.005, 60
    u0 = phased_gaussian(n, 1.5, (0.9, 1.1, 0.8), (0.5, -0.4, 0.3))
    ref = oracle.run_complex(u0, dt, steps)
    with kg.Solver(n, dt, precision=kg.KG_FP32, complex_field=True) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
    assert rel_l2(u, ref["u"]) <= 1e-4
    assert abs(E - ref["energy"][steps]) <= 1e-4 * abs(ref["energy"][steps])


def test_discrete_charge_is_conserved(kg):
    n, dt, steps = 32, 0.01, 200
    u0 = phased_gaussian(n, 1.1, (1.0, 0.8, 1.2), (0.6, -0.3, 0.18))
    with kg.Solver(n, dt, complex_field=True) as s:
        s.set_state(u0, 0.4j * u0)
        c0 = spectral_charge(n, dt, s.spectrum(1), s.spectrum(0))
        s.step(steps)
        c1 = spectral_charge(n, dt, s.spectrum(1), s.spectrum(0))
    assert abs(c0) > 1.0
    assert abs(c1 - c0) <= 1e-12 * abs(c0)


def test_linear_energy_is_conserved(kg):
    n, dt, steps = 24, 0.02, 150
    u0 = phased_gaussian(n, 0.9, (0.9, 1.2, 1.0), (0.3, 0.4, -0.2))
    with kg.Solver(n, dt, linear_only=True, complex_field=True) as s:
        s.set_state(u0, 0.2j * u0)
        E0, _ = s.energy()
        s.step(steps)
        elin, _, _ = s.records(0, steps)
        E1, _ = s.energy()
    assert np.abs(elin - E0).max() <= 1e-12 * abs(E0)
    assert abs(E1 - E0) <= 1e-12 * abs(E0)


def test_blowup_step_matches_oracle(kg):
    n, dt, thr = 32, 0.01, 20.0
    u0 = phased_gaussian(n, 3.0, (1.0, 1.0, 1.0), (0.3, 0.0, 0.0))
    ref = oracle.run_complex(u0, dt, 2000, threshold=thr)
    assert ref["blowup_step"] > 0
    with kg.Solver(n, dt, blowup_threshold=thr, complex_field=True) as s:
        s.set_state(u0)
        st, done = s.step(2000)
        _, blown, bstep = s.stats()
    assert st == kg.KG_BLOWUP and blown
    assert bstep == ref["blowup_step"] == done


@pytest.mark.parametrize("precision", [0, 1])
def test_save_load_and_plan_mismatch(kg, precision):
    n, dt = 24, 0.01
    u0 = phased_gaussian(n, 1.2, (1.0, 0.9, 1.1), (0.5, 0.2, -0.3))
    with kg.Solver(n, dt, precision=precision, complex_field=True) as s:
        s.set_state(u0)
        s.step(10)
        buf = s.save()
        s.step(15)
        ua = s.u()
    with kg.Solver(n, dt, precision=precision, complex_field=True) as s:
        s.load(buf)
        s.step(15)
        ub = s.u()
    assert np.array_equal(ua, ub)
    with kg.Solver(n, dt, precision=precision) as s:  # a real-field plan refuses a complex state
        with pytest.raises(kg.KGError):
            s.load(buf)
    with kg.Solver(n, dt, complex_field=True) as s:
        with pytest.raises(TypeError):
            s.set_state(u0.real.copy())


def test_slab_chain_is_bitwise_independent_of_slab_count(kg, monkeypatch):
    """256^3 complex FP64 (268 MB) is above the cache size: stepped in slabs
    by default; one slab gives the same bits."""
    import torch
    n, dt = 256, 0.002
    u0 = phased_gaussian(n, 1.5, (1.0, 0.9, 1.1), (0.4, -0.2, 0.3))
    out = []
    for mb in ("0", None):
        if mb is None:
            monkeypatch.delenv("KG_SLAB_MB", raising=False)
        else:
            monkeypatch.setenv("KG_SLAB_MB", mb)
        with kg.Solver(n, dt, complex_field=True) as s:
            s.set_state(torch.from_numpy(u0).cuda())
            s.step(8)
            s.step(3)
            out.append((s.u(), s.energy()[0]))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def device_wave(torch, n, mode, phase, amp):
    """amp exp(i (k.x + phase)) on the grid, built on the GPU, [z][y][x]."""
    x = torch.tensor(ki.axis(n), device="cuda", dtype=torch.float64)
    k = [2 * np.pi * m / L for m in mode]
    ph = (k[2] * x)[:, None, None] + (k[1] * x)[None, :, None] + (k[0] * x)[None, None, :]
    return (amp * torch.exp(1j * (ph + phase))).contiguous()


@pytest.mark.parametrize("precision,dealias,mode,tol", [
    (0, False, (3, -2, 5), 1e-11),       # nonlinear frequency, FP64
    (1, False, (3, -2, 5), 2e-5),        # FP32 storage of the same wave
    (0, True, (171, 4, -2), 1e-11),      # outside the kept box: linear frequency
    (0, True, (170, -170, 9), 1e-11)])   # on the box edge (512 // 3 = 170): nonlinear
def test_plane_wave_at_512(kg, precision, dealias, mode, tol):
    """The benchmark's grid and launch configuration (slab chain on two
    streams, graph replays): a complex plane wave advances by exactly theta
    per step."""
    import torch
    n, dt, steps, amp = 512, 0.005, 24, 0.8
    al, be = coeffs(n, dt, mode)
    inside = not dealias or max(abs(m) for m in mode) <= n // 3
    th = np.arccos((al + (be * amp * amp if inside else 0.0)) / 2)
    with kg.Solver(n, dt, precision=precision, complex_field=True, dealias=dealias) as s:
        s.set_state(device_wave(torch, n, mode, 0.0, amp), device_wave(torch, n, mode, th, amp),
                    kg.KG_INIT_TWO_LEVEL)
        s.step(steps)
        out = torch.empty((n, n, n), dtype=torch.complex128, device="cuda")
        s.u(out)
        err = (out - device_wave(torch, n, mode, -steps * th, amp)).abs().max().item()
        _, _, maxu = s.records(0, steps)
    assert err <= tol * amp
    assert np.allclose(maxu, amp, rtol=10 * tol)


def test_real_data_as_complex_field_at_512(kg):
    """The 512^3 benchmark Gaussian stepped as a complex field matches the
    real path (full-spectrum vs half-spectrum kernels) after 20 steps."""
    import torch
    n, dt, steps = 512, 0.005, 20
    x = torch.tensor(ki.axis(n), device="cuda", dtype=torch.float64)
    r2 = (x * x)[:, None, None] + (x * x)[None, :, None] + (x * x)[None, None, :]
    u0 = (1.5 * torch.exp(-r2)).contiguous()
    outs = []
    for cf in (False, True):
        with kg.Solver(n, dt, complex_field=cf) as s:
            s.set_state(u0.to(torch.complex128).contiguous() if cf else u0)
            s.step(steps)
            out = torch.empty((n, n, n), dtype=torch.complex128 if cf else torch.float64,
                              device="cuda")
            s.u(out)
            outs.append((out, s.energy()[0]))
    (ur, Er), (uc, Ec) = outs
    scale = ur.abs().max().item()
    assert (uc.real - ur).abs().max().item() <= 1e-12 * scale
    assert uc.imag.abs().max().item() <= 1e-12 * scale
    assert abs(Ec - Er) <= 1e-12 * abs(Er)


@pytest.mark.parametrize("precision", [0, 1])
def test_kernel_bytes_and_times_of_complex_plans(kg, precision):
    """The algorithmic bytes the bench divides by: one sweep is every stored
    spectral value once (n^3 for a complex field, n^2 (n/2+1) for a real one);
    the z pass moves 5 sweeps in FP64 and 6 in FP32, the others 2."""
    n = 64
    esz = 16 if precision == 0 else 8
    for cf, values in ((True, n ** 3), (False, n * n * (n // 2 + 1))):
        with kg.Solver(n, 0.01, precision=precision, complex_field=cf) as s:
            sweep = values * esz
            assert kg.kg_kernel_bytes(s.plan, 2) == (5 if precision == 0 else 6) * sweep
            for k in (0, 1, 3):
                assert kg.kg_kernel_bytes(s.plan, k) == 2 * sweep
            z, y, x = ki.mesh(n, L)
            u0 = ki.gaussian(n, 0.5) * (np.exp(0.5j * x) if cf else 1.0)
            s.set_state(u0)
            kg.kg_step(s.plan, 3, kg.KG_STEP_TIMED)
            ms, steps = kg.kg_kernel_times(s.plan)
            assert steps == 3 and all(t > 0 for t in ms)
