"""Parity of the GPU stepper (through the C-ABI) with the oracle and with the
closed forms that pin it: eq. (2) of Sec. 1.1.2 and the energy of Sec. 1.1.

Tolerances.  The FP64 target is a relative L2 error of at most 1e-11 after
100 steps.  Closed forms that the scheme reproduces exactly (discrete plane
wave, exact linear energy conservation) are held to 1e-12 as in the oracle
pins; bitwise properties (determinism, checkpoint resume) are exact.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle

pytestmark = pytest.mark.gpu

L = ki.BOX


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def omega_of_mode(mode):
    k = 2 * np.pi * np.asarray(mode, float) / L
    return np.sqrt(1.0 + np.sum(k * k))


def test_small_config_matches_oracle(kg):
    """32^3, u0 = 0.1 exp(-|x|^2), u_t0 = 0, dt = 0.01, 100 steps."""
    n, dt, steps = 32, 0.01, 100
    u0 = ki.gaussian(n, 0.1)
    ref = oracle.run(u0, dt, steps)
    with kg.Solver(n, dt) as s:
        s.set_state(u0)
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        u = s.u()
        E, t = s.energy()
        elin, q4, maxu = s.records(0, steps)
        vn = s.spectrum(0)
    assert rel_l2(u, ref["u"]) <= 1e-11
    assert abs(t - (steps - 0.5) * dt) < 1e-12
    assert abs(E - ref["energy"][steps]) <= 1e-11 * abs(ref["energy"][steps])
    assert np.allclose(maxu, ref["maxu"][:steps], rtol=1e-11, atol=0)
    assert np.allclose(q4, ref["q4"][:steps], rtol=1e-10, atol=0)
    _, vc = oracle.state(u0, dt, steps)
    assert np.abs(vn - vc[:, :, :n // 2 + 1]).max() <= 1e-11 * np.abs(vc).max()


@pytest.mark.parametrize("n,A,sigma,steps", [(64, 1.5, (1.0, 1.0, 1.0), 100),
                                             (16, 1.2, (0.9, 1.1, 1.4), 100),
                                             (48, 2.0, (0.7, 1.3, 1.0), 100),
                                             (96, 1.5, (0.6, 0.9, 1.2), 60),
                                             (128, 1.0, (0.8, 1.0, 1.3), 30)])
def test_nonlinear_gaussian_matches_oracle(kg, n, A, sigma, steps):
    dt = 0.005
    u0 = ki.gaussian(n, A, sigma) + ki.gaussian(n, 0.3, (1.0, 1.0, 1.0), center=(2.0, -1.0, 0.5))
    ref = oracle.run(u0, dt, steps)
    with kg.Solver(n, dt) as s:
        s.set_state(u0)
        s.step(steps)
        u = s.u()
        E, _ = s.energy()
    assert rel_l2(u, ref["u"]) <= 1e-11
    assert abs(E - ref["energy"][steps]) <= 1e-11 * abs(ref["energy"][steps])


def test_velocity_and_two_level_starts(kg):
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 0.8, (1.0, 1.2, 0.9))
    ut0 = ki.gaussian(n, 0.5, (1.1, 0.8, 1.0), center=(1.0, 0.0, -1.0))
    um1 = ki.gaussian(n, 0.79, (1.0, 1.2, 0.9))
    for mode, aux in ((oracle.INIT_VELOCITY, ut0), (oracle.INIT_TWO_LEVEL, um1)):
        ref = oracle.run(u0, dt, 20, mode=mode, aux=aux)
        with kg.Solver(n, dt) as s:
            s.set_state(u0, aux, mode)
            E0, _ = s.energy()
            s.step(20)
            u = s.u()
        assert abs(E0 - ref["energy"][0]) <= 1e-12 * abs(ref["energy"][0])
        assert rel_l2(u, ref["u"]) <= 1e-11


@pytest.mark.parametrize("n", [16, 32, 512])
def test_discrete_plane_wave(kg, n):
    """u^m = cos(k.x - m th), tan(th/2) = omega dt/2, solves the linear scheme
    exactly; k = (1, 2, 0) (mode (4, 8, 0)) on the 8 pi box."""
    dt, steps = 0.01, 100 if n < 512 else 40
    mode = (4, 8, 0) if n >= 32 else (1, 2, 3)
    w = omega_of_mode(mode)
    th = 2 * np.arctan(w * dt / 2)
    with kg.Solver(n, dt, linear_only=True) as s:
        s.set_state(ki.plane_wave(n, mode), ki.plane_wave(n, mode, th), kg.KG_INIT_TWO_LEVEL)
        E0, _ = s.energy()
        s.step(steps)
        u = s.u()
        E1, _ = s.energy()
    assert rel_l2(u, ki.plane_wave(n, mode, -steps * th)) <= 1e-12
    assert abs(E1 - E0) <= 1e-12 * abs(E0)


def test_linear_energy_is_conserved(kg):
    n, dt, steps = 64, 0.01, 200
    with kg.Solver(n, dt, linear_only=True) as s:
        s.set_state(ki.gaussian(n, 0.7, (0.9, 1.1, 1.3)))
        E0, _ = s.energy()
        s.step(steps)
        elin, q4, _ = s.records(0, steps)
        E1, _ = s.energy()
    assert np.abs(elin - E0).max() <= 1e-12 * abs(E0)
    assert abs(E1 - E0) <= 1e-12 * abs(E0)


@pytest.mark.parametrize("n", [8, 512])
def test_uniform_data_blows_up_at_the_oracle_step(kg, n):
    """Uniform a = 1.5 reduces eq. (1) to y'' + y = y^3, which blows up; the
    first level above 1e3 is step 145 at dt = 0.01 (the oracle's step)."""
    dt = 0.01
    ref = oracle.run(ki.uniform(8, 1.5), dt, 300, threshold=1e3)
    assert ref["blowup_step"] == 145
    with kg.Solver(n, dt, blowup_threshold=1e3) as s:
        s.set_state(ki.uniform(n, 1.5))
        st, done = s.step(300)
        steps, blown, bstep = s.stats()
        _, _, maxu = s.records(0, bstep + 1)
    assert st == kg.KG_BLOWUP and blown and bstep == 145 and done == 145
    assert np.allclose(maxu, ref["maxu"][:146], rtol=1e-11)


def test_nonfinite_input_is_a_blowup(kg):
    u0 = ki.gaussian(16, 0.1)
    u0[3, 4, 5] = np.nan
    with kg.Solver(16, 0.01, blowup_threshold=1e3) as s:
        s.set_state(u0)
        st, done = s.step(5)
        assert st == kg.KG_BLOWUP and done == 0
        assert s.stats()[2] == 0


def test_gaussian_blowup_matches_oracle(kg):
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 4.0, (1.0, 1.2, 0.9))
    ref = oracle.run(u0, dt, 400, threshold=1e3)
    assert ref["blowup_step"] > 0
    with kg.Solver(n, dt, blowup_threshold=1e3) as s:
        s.set_state(u0)
        st, done = s.step(400)
        assert st == kg.KG_BLOWUP and s.stats()[2] == ref["blowup_step"]


def test_determinism_and_checkpoint(kg):
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.5, (0.9, 1.1, 1.3))
    with kg.Solver(n, dt) as a, kg.Solver(n, dt) as b:
        a.set_state(u0)
        b.set_state(u0)
        a.step(100)
        b.step(50)
        blob = b.save()
        b.set_state(ki.gaussian(n, 0.3))  # clobber, then resume
        b.step(3)
        b.load(blob)
        b.step(50)
        ua, ub = a.u(), b.u()
        Ea, Eb = a.energy(), b.energy()
        assert np.array_equal(ua, ub)
        assert Ea == Eb
        sa, sb = a.spectrum(1), b.spectrum(1)
        assert np.array_equal(sa, sb)


@pytest.mark.parametrize("precision", [0, 1])
def test_slab_chain_is_bitwise_independent_of_slab_count(kg, monkeypatch, precision):
    """Fields above the cache size step their y-inverse / x / y-forward chain
    slab by slab of z planes, in captured graphs on one or two streams; every
    line sees the same arithmetic, so one slab, the default slabs and many
    ragged slabs, on either schedule, agree bitwise (384^3: 2 default slabs in
    FP64; 10 slabs of 40 planes, the last of 24).  Eight steps replay a graph,
    the rest run eagerly, around an energy() call that rebuilds the field."""
    n, dt = 384, 0.005
    u0 = ki.gaussian(n, 1.2, (0.8, 1.0, 1.3))
    out = {}
    for mb in ("0", None, "50"):
        for streams in ("1", "2"):
            if mb is None:
                monkeypatch.delenv("KG_SLAB_MB", raising=False)
            else:
                monkeypatch.setenv("KG_SLAB_MB", mb)
            monkeypatch.setenv("KG_SLAB_STREAMS", streams)
            with kg.Solver(n, dt, precision=precision) as s:
                s.set_state(u0)
                s.step(8)
                E = s.energy()
                s.step(3)
                out[(mb, streams)] = (s.u(), E, s.spectrum(0), s.records(0, 11))
    ref = out[("0", "1")]
    for key, got in out.items():
        assert np.array_equal(got[0], ref[0]), key
        assert got[1] == ref[1], key
        assert np.array_equal(got[2], ref[2]), key
        for a, b in zip(got[3], ref[3]):
            assert np.array_equal(a, b), key


def test_first_step_at_512_sampled_modes(kg):
    """Full size: v^0 and v^1 at sampled modes against direct DFT sums."""
    n, dt = 512, 0.005
    u0 = ki.gaussian(n, 1.5, (0.9, 1.1, 1.3), center=(0.2, -0.4, 0.3))
    with kg.Solver(n, dt) as s:
        s.set_state(u0)
        s.step(1)
        v1 = s.spectrum(0)
        v0 = s.spectrum(1)
    modes = [(0, 0, 0), (1, 0, 0), (0, 3, 0), (0, 0, 5), (7, 11, 13), (256, 256, 256),
             (40, 500, 3), (128, 1, 400)]
    r0, r1 = oracle.first_step_modes(u0, dt, modes)
    for (ix, iy, iz), a, b in zip(modes, r0, r1):
        assert abs(v0[iz, iy, ix] - a) <= 1e-12 * np.abs(r0).max()
        assert abs(v1[iz, iy, ix] - b) <= 1e-12 * np.abs(r1).max()


def test_uniform_recurrence_at_512(kg):
    """Uniform data at full size follows the oracle's uniform run.  Both sides
    round every step; the difference grows like steps * log2(M) * eps
    (50 * 27 * 1.1e-16 ~ 1.5e-13 relative), so 1e-12 relative is the bound."""
    n, dt, steps = 512, 0.005, 50
    ref = oracle.run(ki.uniform(8, 0.5), dt, steps)
    with kg.Solver(n, dt) as s:
        s.set_state(ki.uniform(n, 0.5))
        s.step(steps)
        u = s.u()
    assert np.ptp(u) <= 1e-12
    assert abs(u[0, 0, 0] - ref["u"][0, 0, 0]) <= 1e-12 * abs(ref["u"][0, 0, 0])


def test_graph_replays_match_single_step_launches(kg):
    """Runs of >= 8 steps replay captured graphs; single steps launch eagerly.
    Both paths must give the same bits, across several replays with eager work
    and synchronisation in between."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.5, (0.9, 1.1, 1.3))
    with kg.Solver(n, dt) as a, kg.Solver(n, dt) as b:
        a.set_state(u0)
        b.set_state(u0)
        for rep in range(3):
            for _ in range(16):
                a.step(1)
            b.step(16)
            assert a.stats()[0] == b.stats()[0] == 16 * (rep + 1)
            assert np.array_equal(a.u(), b.u())
            assert a.energy() == b.energy()
        assert np.array_equal(a.records(0, 48)[0], b.records(0, 48)[0])


def test_stepping_after_a_blowup_and_argument_checks(kg):
    """After a blow-up the counter stays at the blown level, further steps and
    the energy report KG_BLOWUP; zero steps are a no-op, negative ones an
    error."""
    with kg.Solver(8, 0.01, blowup_threshold=1e3) as s:
        s.set_state(ki.uniform(8, 1.5))
        st, done = s.step(0)
        assert st == kg.KG_OK and done == 0
        with pytest.raises(kg.KGError) as e:
            s.step(-1)
        assert e.value.status == kg.KG_E_INVALID
        st, done = s.step(200)
        assert st == kg.KG_BLOWUP and done == 145
        st, done = s.step(20)  # graphs and single steps alike do nothing now
        assert st == kg.KG_BLOWUP and done == 145
        assert s.stats() == (145, True, 145)
        assert np.isnan(s.energy()[0])


def test_disabled_threshold_still_stops_at_nonfinite_values(kg):
    """threshold <= 0 disables the max|u| test, but a level with a non-finite
    value still ends the run, at the oracle's level."""
    dt = 0.01
    ref = oracle.run(ki.uniform(8, 1.5), dt, 300, threshold=0.0)
    assert ref["blowup_step"] > 145
    with kg.Solver(8, dt, blowup_threshold=0.0) as s:
        s.set_state(ki.uniform(8, 1.5))
        st, done = s.step(300)
    assert st == kg.KG_BLOWUP and done == ref["blowup_step"]


def test_records_keep_the_last_65536_levels(kg):
    n, steps = 8, 65536 + 40
    with kg.Solver(n, 0.01, linear_only=True) as s:
        s.set_state(ki.gaussian(n, 0.1))
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        elin, q4, maxu = s.records(40, 65536)
        assert np.all(np.isfinite(elin)) and np.all(maxu > 0)
        # eq. (2) conserves the linear energy exactly; rounding over 65 576 steps
        assert np.abs(elin - elin[0]).max() <= 1e-9 * abs(elin[0])
        with pytest.raises(kg.KGError) as e:
            s.records(39, 1)
        assert e.value.status == kg.KG_E_INVALID


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("complex_field", [False, True])
def test_plane_padding_does_not_change_results(kg, monkeypatch, precision, complex_field):
    """The z-plane padding of the working field only moves addresses: runs
    with 0, the default and 4 KiB of padding agree bit for bit."""
    n, dt, steps = 48, 0.005, 30
    u0 = ki.gaussian(n, 1.8, (0.7, 1.2, 0.9))
    if complex_field:
        z, y, x = ki.mesh(n, L)
        u0 = u0 * np.exp(0.4j * x)
    out = []
    for pad in ("0", None, "4096"):
        if pad is None:
            monkeypatch.delenv("KG_PLANE_PAD", raising=False)
        else:
            monkeypatch.setenv("KG_PLANE_PAD", pad)
        with kg.Solver(n, dt, precision=precision, complex_field=complex_field) as s:
            s.set_state(u0)
            s.step(steps)
            out.append((s.u(), s.energy()[0]))
    for u, E in out[1:]:
        assert np.array_equal(u, out[0][0])
        assert E == out[0][1]
