"""Pins for the oracle's time stepper (eq. (2) of Sec. 1.1.2) against what the
paper and the mathematics fix: exact discrete and continuous solutions, the
conserved energy of Sec. 1.1, closed forms, symmetries of eq. (1), and eq. (2)
solved directly as a dense linear system on a tiny grid.
"""
import numpy as np
import pytest
from scipy import integrate, special

import kg_inputs as ki
import oracle

L = ki.BOX


def omega_of_mode(mode, Ls=(L, L, L)):
    k = 2 * np.pi * np.asarray(mode, float) / np.asarray(Ls, float)
    return np.sqrt(1.0 + np.sum(k * k))


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------
# Linear equation (cubic term off): exact discrete plane wave
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,mode,Ls", [
    (32, (4, 8, 0), (L, L, L)),        # physical k = (1, 2, 0)
    (32, (1, 2, 0), (L, L, L)),
    ((16, 24, 12), (3, -5, 2), (L, 0.75 * L, 0.5 * L)),  # anisotropic grid and box
    (16, (8, 0, 0), (L, L, L)),        # the Nyquist mode
])
def test_discrete_plane_wave_is_exact(n, mode, Ls):
    """u^n = cos(k.x - n theta) with tan(theta/2) = omega dt / 2 solves the
    linear part of eq. (2) exactly: substituting it gives
    (2 cos th - 2)/dt^2 + omega^2 (2 cos th + 2)/4 = 0."""
    dt = 0.01
    w = omega_of_mode(mode, Ls)
    th = 2 * np.arctan(w * dt / 2)
    u0 = ki.plane_wave(n, mode, 0.0, Ls)
    um1 = ki.plane_wave(n, mode, th, Ls)
    r = oracle.run(u0, dt, 100, L=Ls, linear_only=True, mode=oracle.INIT_TWO_LEVEL, aux=um1)
    exact = ki.plane_wave(n, mode, -100 * th, Ls)
    assert rel_l2(r["u"], exact) <= 1e-12
    exact_prev = ki.plane_wave(n, mode, -99 * th, Ls)
    assert rel_l2(r["u_prev"], exact_prev) <= 1e-12


def test_plane_wave_converges_to_pde_solution_at_second_order():
    """u = cos(k.x - omega t), omega^2 = |k|^2 + 1, solves eq. (1) without the
    cubic term; the scheme's phase error after time t is about t omega^3 dt^2/12."""
    mode = (4, 8, 0)
    w = omega_of_mode(mode)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        nsteps = int(round(1.0 / dt))
        u0 = ki.plane_wave(32, mode)
        ut0 = w * ki.plane_wave(32, mode, fn=np.sin)
        r = oracle.run(u0, dt, nsteps, linear_only=True, aux=ut0)
        exact = ki.plane_wave(32, mode, -w * nsteps * dt)
        errs.append(rel_l2(r["u"], exact))
        # phase error t omega^3 dt^2 / 12 plus the O(dt^2) start-up term below
        assert errs[-1] <= 2.0 * (1.0 * w ** 3 * dt * dt / 12)
    assert 3.9 < errs[0] / errs[1] < 4.1 and 3.9 < errs[1] / errs[2] < 4.1


@pytest.mark.parametrize("dt", [0.01, 0.05])
def test_velocity_start_discrete_closed_form(dt):
    """Start from u0 = cos(k.x), u_t0 = omega sin(k.x).  The cos and sin
    amplitudes each follow the two-term recurrence of the linear scheme, whose
    solutions are cos(n th), sin(n th) with cos th = alpha/2; the symmetric start
    gives them the levels cos(th) and -omega dt at n = -1, hence exactly
    u^n = cos(k.x - n th) + a sin(n th) sin(k.x),  a = omega^2 dt^2 / 4."""
    mode = (4, 8, 0)
    w = omega_of_mode(mode)
    th = 2 * np.arctan(w * dt / 2)
    a = w * w * dt * dt / 4
    n = 37
    r = oracle.run(ki.plane_wave(32, mode), dt, n, linear_only=True,
                   aux=w * ki.plane_wave(32, mode, fn=np.sin))
    expect = ki.plane_wave(32, mode, -n * th) + a * np.sin(n * th) * ki.plane_wave(32, mode, fn=np.sin)
    assert np.abs(r["u"] - expect).max() <= 1e-12


# --------------------------------------------------------------------------
# Spatially uniform data: eq. (1) reduces to y'' + y = y^3
# --------------------------------------------------------------------------

def cd_solution(a, t):
    """y'' + y = y^3, y(0) = a < 1, y'(0) = 0: y = a cd(lam t | m) with
    lam^2 = 1 - a^2/2 and m = a^2/(2 - a^2) (Jacobi elliptic cd = cn/dn)."""
    lam = np.sqrt(1 - a * a / 2)
    m = a * a / (2 - a * a)
    sn, cn, dn, _ = special.ellipj(lam * t, m)
    return a * cn / dn


def test_cd_closed_form_solves_the_ode():
    a = 0.5
    sol = integrate.solve_ivp(lambda t, y: [y[1], y[0] ** 3 - y[0]], (0, 10), [a, 0.0],
                              rtol=1e-12, atol=1e-14, dense_output=True)
    t = np.linspace(0, 10, 41)
    assert np.abs(sol.sol(t)[0] - cd_solution(a, t)).max() < 1e-9


def test_uniform_data_matches_ode_at_second_order():
    a, T = 0.5, 10.0
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        nsteps = int(round(T / dt))
        r = oracle.run(ki.uniform(8, a), dt, nsteps)
        assert np.ptp(r["u"]) <= 1e-13  # stays uniform
        errs.append(abs(r["u"][0, 0, 0] - cd_solution(a, T)))
    assert errs[0] < 2e-5
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


def blowup_time(a, Y):
    """Time for y'' + y = y^3, y(0) = a > 1, y'(0) = 0 to reach Y:
    y'^2 = (y^2 - a^2)(y^2 + a^2 - 2)/2; substitute y = a + s^2."""
    def f(s):
        y = a + s * s
        return 2.0 / np.sqrt((2 * a + s * s) * (y * y + a * a - 2) / 2)
    return integrate.quad(f, 0, np.sqrt(Y - a), limit=200, epsabs=1e-13, epsrel=1e-13)[0]


def test_blowup_step_tracks_the_ode_blowup_time():
    """Uniform a = 1.5 blows up; the first level with max|u| > 1e3 times dt
    approaches t(1e3) from above as dt shrinks."""
    a, Y = 1.5, 1e3
    tb = blowup_time(a, Y)
    assert abs(tb - 1.4408) < 1e-4
    gaps = []
    for dt in (0.01, 0.005, 0.0025):
        r = oracle.run(ki.uniform(8, a), dt, int(2 / dt), threshold=Y)
        n = r["blowup_step"]
        assert n > 0
        assert r["maxu"][n] > Y and r["maxu"][n - 1] <= Y
        assert np.all(np.isnan(r["energy"][n + 1:]))
        gaps.append(n * dt - tb)
    assert all(0 < g < dt for g, dt in zip(gaps, (0.01, 0.005, 0.0025)))
    assert gaps[0] > gaps[1] > gaps[2]


def test_nonfinite_data_is_a_blowup_at_step_zero():
    u0 = ki.gaussian(8)
    u0[1, 2, 3] = np.nan
    r = oracle.run(u0, 0.01, 5, threshold=1e3)
    assert r["blowup_step"] == 0


# --------------------------------------------------------------------------
# Energy (Sec. 1.1)
# --------------------------------------------------------------------------

def gaussian_energy(A, s):
    """E of u = A exp(-sum x_i^2/s_i^2), u_t = 0 on R^3:
    int u^2 = A^2 (pi/2)^{3/2} S, int |grad u|^2 = A^2 (pi/2)^{3/2} S sum s_i^-2,
    int u^4 = A^4 (pi/4)^{3/2} S, S = sx sy sz."""
    S = s[0] * s[1] * s[2]
    return np.pi ** 1.5 * S * (A * A * (1 + sum(1 / si ** 2 for si in s)) / 2 ** 2.5 - A ** 4 / 32)


@pytest.mark.parametrize("n,A,s", [(64, 0.1, (1, 1, 1)), (64, 1.5, (1, 1, 1)),
                                   (96, 1.0, (0.8, 1.0, 1.25))])
def test_initial_energy_matches_gaussian_closed_form(n, A, s):
    """Sampled on the grid, the Gaussian's spectrum is resolved to ~1e-10 at
    h = 8 pi / 64 for s = 1 (and at 96 points for s = 0.8); the start adds O(dt^2)."""
    assert abs(gaussian_energy(0.1, (1, 1, 1)) - 0.0393566) < 1e-7
    r = oracle.run(ki.gaussian(n, A, s), 1e-4, 0)
    E = gaussian_energy(A, s)
    assert abs(r["energy"][0] - E) <= 1e-6 * abs(E)


def test_linear_energy_is_exactly_conserved():
    r = oracle.run(ki.gaussian(32, 0.5, (0.9, 1.1, 1.3)), 0.01, 100, linear_only=True)
    E = r["energy"]
    assert np.abs(E - E[0]).max() <= 1e-12 * abs(E[0])


def test_nonlinear_energy_drift_is_second_order():
    drifts = []
    for dt in (0.01, 0.005, 0.0025):
        r = oracle.run(ki.gaussian(32, 1.5), dt, int(round(0.5 / dt)))
        E = r["energy"]
        drifts.append(np.abs(E - E[0]).max() / abs(E[0]))
    assert drifts[0] < 1e-2
    assert 3.5 < drifts[0] / drifts[1] < 4.5 and 3.5 < drifts[1] / drifts[2] < 4.5


def test_time_convergence_of_nonlinear_gaussian_run():
    T = 0.4
    us = []
    for dt in (0.01, 0.005, 0.0025):
        us.append(oracle.run(ki.gaussian(24, 1.5, (0.9, 1.1, 1.3)), dt, int(round(T / dt)))["u"])
    e1 = np.linalg.norm(us[0] - us[1])
    e2 = np.linalg.norm(us[1] - us[2])
    assert 3.6 < e1 / e2 < 4.4


# --------------------------------------------------------------------------
# Symmetries of eq. (1) on the periodic grid
# --------------------------------------------------------------------------

def lumpy(n):
    return ki.gaussian(n, 1.2, (0.9, 1.1, 1.4)) + \
        ki.gaussian(n, 0.7, (1.3, 0.8, 1.0), center=(2.0, -1.5, 3.0))


def test_reflection_symmetry():
    """x_{N-j} = -x_j on the grid, so reflecting the data reflects the solution."""
    u0 = lumpy(16)
    base = oracle.run(u0, 0.01, 20)["u"]
    for ax in range(3):
        refl = np.roll(np.flip(u0, axis=ax), 1, axis=ax)
        got = oracle.run(refl, 0.01, 20)["u"]
        expect = np.roll(np.flip(base, axis=ax), 1, axis=ax)
        assert np.abs(got - expect).max() <= 1e-12


def test_axis_permutation_and_translation():
    u0 = lumpy(16)
    base = oracle.run(u0, 0.01, 20)["u"]
    perm = np.ascontiguousarray(np.transpose(u0, (2, 0, 1)))
    got = oracle.run(perm, 0.01, 20)["u"]
    assert np.abs(got - np.transpose(base, (2, 0, 1))).max() <= 1e-12
    sh = np.roll(u0, (3, -2, 5), axis=(0, 1, 2))
    got = oracle.run(sh, 0.01, 20)["u"]
    assert np.abs(got - np.roll(base, (3, -2, 5), axis=(0, 1, 2))).max() <= 1e-12


# --------------------------------------------------------------------------
# Eq. (2) solved directly, as written, on a tiny grid
# --------------------------------------------------------------------------

def dense_laplacian(nx, ny, nz, Ls):
    """The spectral Laplacian as a dense M x M real matrix, from the brute-force
    3D DFT matrix (symbol -|k|^2, k = 2 pi m / L, m the signed mode number)."""
    M = nx * ny * nz
    jz, jy, jx = [g.ravel() for g in np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                                                   indexing="ij")]
    ph = (np.outer(jx, jx) % nx) / nx + (np.outer(jy, jy) % ny) / ny + (np.outer(jz, jz) % nz) / nz
    F = np.exp(-2j * np.pi * ph)
    def m(i, n):
        return np.where(i <= n // 2, i, i - n)
    k2 = (2 * np.pi * m(jx, nx) / Ls[0]) ** 2 + (2 * np.pi * m(jy, ny) / Ls[1]) ** 2 + \
        (2 * np.pi * m(jz, nz) / Ls[2]) ** 2
    lap = (F.conj().T @ (-k2[:, None] * F)) / M
    assert np.abs(lap.imag).max() < 1e-9
    return lap.real


def test_eq2_as_dense_linear_solve():
    """(u+ - 2u + u-)/dt^2 - Lap (u+ + 2u + u-)/4 + (u+ + 2u + u-)/4 = u^3,
    solved for u+ with a dense solver in physical space, five steps."""
    nx, ny, nz = 6, 4, 8
    Ls = (L, 0.6 * L, 1.3 * L)
    dt = 0.05
    rng = np.random.default_rng(11)
    shape = (nz, ny, nx)
    um1 = 0.8 * ki.gaussian((nx, ny, nz), 1.0, (5.0, 3.0, 6.0), Ls) + 0.1 * rng.standard_normal(shape)
    u0 = um1 + 0.05 * rng.standard_normal(shape)
    lap = dense_laplacian(nx, ny, nz, Ls)
    I = np.eye(nx * ny * nz)
    A = I / dt ** 2 + (I - lap) / 4
    up, uc = um1.ravel(), u0.ravel()
    for _ in range(5):
        rhs = uc ** 3 + (2 * uc - up) / dt ** 2 - (I - lap) @ (2 * uc + up) / 4
        up, uc = uc, np.linalg.solve(A, rhs)
    r = oracle.run(u0, dt, 5, L=Ls, mode=oracle.INIT_TWO_LEVEL, aux=um1)
    assert np.abs(r["u"].ravel() - uc).max() <= 1e-12 * np.abs(uc).max()
    assert np.abs(r["u_prev"].ravel() - up).max() <= 1e-12 * np.abs(up).max()


def test_direct_sum_first_step_matches_the_fft_stepper():
    """The sampled-mode entry (direct DFT sums) and the FFT stepper are two
    independent routes to v^0 and v^1."""
    u0 = lumpy(16)
    modes = [(0, 0, 0), (1, 2, 3), (8, 5, 15), (3, 0, 8), (15, 15, 1)]
    for lin in (False, True):
        v0, v1 = oracle.first_step_modes(u0, 0.01, modes, linear_only=lin)
        vp, vc = oracle.state(u0, 0.01, 1, linear_only=lin)
        for (ix, iy, iz), a, b in zip(modes, v0, v1):
            assert abs(a - vp[iz, iy, ix]) <= 1e-13 * np.abs(vp).max()
            assert abs(b - vc[iz, iy, ix]) <= 1e-13 * np.abs(vc).max()
