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
    the rest single-step graphs, around an energy() call that rebuilds the
    field."""
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


def test_graph_replays_match_eager_launches(kg):
    """Steps replay captured graphs (8-step and single-step ones); timed steps
    launch every kernel eagerly.  All three must give the same bits, across
    several replays with eager work and synchronisation in between."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.5, (0.9, 1.1, 1.3))
    with kg.Solver(n, dt) as a, kg.Solver(n, dt) as b, kg.Solver(n, dt) as c:
        for s in (a, b, c):
            s.set_state(u0)
        for rep in range(3):
            for _ in range(16):
                a.step(1)
            b.step(16)
            kg.kg_step(c.plan, 16, kg.KG_STEP_TIMED)
            assert a.stats()[0] == b.stats()[0] == c.stats()[0] == 16 * (rep + 1)
            assert np.array_equal(a.u(), b.u()) and np.array_equal(a.u(), c.u())
            assert a.energy() == b.energy() == c.energy()
        assert np.array_equal(a.records(0, 48)[0], b.records(0, 48)[0])
        assert np.array_equal(a.records(0, 48)[0], c.records(0, 48)[0])


def test_energy_series_and_max_abs_u_match_oracle(kg):
    """kg_energies gives E^{m-1/2} at every level 0..n (the oracle's energy
    array), kg_stats the newest level's max|u|."""
    n, dt, steps = 32, 0.01, 100
    u0 = ki.gaussian(n, 1.3, (0.9, 1.1, 1.3))
    ref = oracle.run(u0, dt, steps)
    with kg.Solver(n, dt) as s:
        s.set_state(u0)
        E0 = s.energies(0, 1)
        assert abs(E0[0] - ref["energy"][0]) <= 1e-12 * abs(ref["energy"][0])
        _, _, _, mx0 = s.stats(max_abs_u=True)
        assert abs(mx0 - ref["maxu"][0]) <= 1e-12 * ref["maxu"][0]
        s.step(steps)
        E = s.energies(0, steps + 1)
        _, _, _, mx = s.stats(max_abs_u=True)
        E_mid = s.energies(40, 21)
        assert s.energy()[0] == E[-1]
        with pytest.raises(kg.KGError) as e:
            s.energies(0, steps + 2)
        assert e.value.status == kg.KG_E_INVALID
    assert np.abs(E - ref["energy"]).max() <= 1e-11 * np.abs(ref["energy"]).max()
    assert np.array_equal(E_mid, E[40:61])
    assert abs(mx - ref["maxu"][steps]) <= 1e-11 * ref["maxu"][steps]


@pytest.mark.parametrize("precision", [0, 1])
def test_levels_after_a_blowup(kg, precision):
    """After a blow-up at level b the blown step has overwritten the level
    before it: kg_get_spectrum(which=1) and kg_get_state's u_prev refuse;
    u^b itself, the energies up to E^{b-1/2} and max|u^b| stay available and
    match the oracle.

    Tolerance at the blown level: the run amplifies a relative perturbation
    of its data by kappa there (measured below with the oracle, data scaled
    by 1 + 1e-13); rounding of ~1e-15 per level accumulates like a random
    walk over the b levels, so u^b is held to 10 kappa 1e-15 sqrt(b).  FP32
    keeps (v, v - v_prev) and rebuilds u^b as v^{b+1} - (v^{b+1} - v^b) in
    float, whose rounding is that of v^{b+1}, many times u^b one step past
    the blow-up: the blown level is then only checked against the record of
    max|u^b| the step itself took, to the FP32 target 1e-4."""
    dt = 0.01
    ref = oracle.run(ki.uniform(8, 1.5), dt, 300, threshold=1e3)
    pert = oracle.run(ki.uniform(8, 1.5 * (1 + 1e-13)), dt, 300, threshold=1e3)
    b = ref["blowup_step"]
    kappa = abs(pert["u"].max() - ref["u"].max()) / ref["u"].max() / 1e-13
    tol_b = max(1e-11, 10 * kappa * 1e-15 * np.sqrt(b))
    with kg.Solver(8, dt, blowup_threshold=1e3, precision=precision) as s:
        s.set_state(ki.uniform(8, 1.5))
        st, done = s.step(300)
        assert st == kg.KG_BLOWUP and abs(done - b) <= precision
        for call in (lambda: s.spectrum(1), lambda: s.state()):
            with pytest.raises(kg.KGError) as e:
                call()
            assert e.value.status == kg.KG_E_INVALID
        _, ub = kg.kg_get_state(s.plan, 8, want_prev=False)
        E = s.energies(0, done + 1)
        steps, blown, bstep, mx = s.stats(max_abs_u=True)
    assert (steps, blown, bstep) == (done, True, done)
    if precision == 1:
        # FP32 may also cross the threshold one level apart from the oracle
        assert abs(mx - np.abs(ub).max()) <= 1e-4 * mx
        return
    assert abs(mx - np.abs(ub).max()) <= 1e-12 * mx
    assert np.abs(ub - ref["u"]).max() <= tol_b * np.abs(ref["u"]).max()
    assert abs(mx - ref["maxu"][b]) <= tol_b * ref["maxu"][b]
    # E is a difference of terms growing like u^4: compare it where max|u| < 3
    # (its terms below ~100 |E|), and its presence up to E^{b-1/2}
    keep = np.flatnonzero(ref["maxu"][:b + 1] < 3.0)
    assert len(keep) > 50 and np.all(np.isfinite(E))
    dE = np.abs(E[keep] - ref["energy"][keep]) / np.abs(ref["energy"][keep])
    assert dE.max() <= 1e-11


@pytest.mark.parametrize("precision", [0, 1])
def test_two_level_restore_from_get_state(kg, precision):
    """(u^{n-1}, u^n) from kg_get_state restart the run with the two-level
    start: the continuation equals the uninterrupted run up to the rounding
    of one transform pair per level.  FP64: a c2r/r2c round trip rounds at
    ~2 log2(M) eps ~ 3e-15 relative, which the 40 further nonlinear steps may
    grow a few times: 3e-14.  FP32 keeps (v, v - v_prev) in float; the
    restart forms v - v_prev from two separately rounded levels, an error
    of eps32 |v| on a difference of size omega dt |v|, so the continuation
    is good to ~eps32 / (omega dt) ~ 1e-5: held to the FP32 target 1e-4."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 0.9, (0.9, 1.1, 1.3))
    with kg.Solver(n, dt, precision=precision) as a, kg.Solver(n, dt, precision=precision) as b:
        a.set_state(u0)
        a.step(60)
        up, uc = a.state()
        assert np.array_equal(uc, a.u())
        b.set_state(uc, up, kg.KG_INIT_TWO_LEVEL)
        Ea, Eb = a.energy()[0], b.energy()[0]
        a.step(40)
        b.step(40)
        ua, ub = a.u(), b.u()
    tol = 3e-14 if precision == 0 else 1e-4
    assert abs(Ea - Eb) <= tol * abs(Ea)
    assert rel_l2(ub, ua) <= tol
    if precision == 0:
        ref = oracle.run(u0, dt, 100)
        assert rel_l2(ub, ref["u"]) <= 1e-11


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


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [48, 512])
def test_persistent_z_pass_matches_tile_kernel(kg, monkeypatch, precision, n):
    """The step's z pass runs as a persistent workgroup-per-CU kernel
    (k_zstep) or, with KG_Z_PERSISTENT=0, one workgroup per tile (k_zpass).
    Both run the same transforms and the same per-mode update, so the levels
    and fields agree bitwise; only the energy's partial sums are grouped
    differently (per workgroup), so energies agree to rounding (1e-14
    relative).  48^3 (radix-3 z lines, ragged tiles) and the benchmark's
    512^3."""
    dt = 0.005
    u0 = ki.gaussian(n, 1.5 if n == 48 else 0.1)
    out = {}
    for persistent in ("1", "0"):
        monkeypatch.setenv("KG_Z_PERSISTENT", persistent)
        with kg.Solver(n, dt, precision=precision) as s:
            s.set_state(u0)
            st, done = s.step(10)
            assert st == kg.KG_OK and done == 10
            elin, q4, maxu = s.records(0, 10)
            out[persistent] = (s.spectrum(0), s.spectrum(1), elin, q4, maxu, s.energy()[0])
    a, b = out["1"], out["0"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])
    assert np.allclose(a[2], b[2], rtol=1e-14, atol=0)
    assert abs(a[5] - b[5]) <= 1e-14 * abs(b[5])


@pytest.mark.parametrize("precision,complex_field", [(0, False), (1, False), (0, True),
                                                     (1, True)])
def test_zero_field_stays_zero(kg, precision, complex_field):
    """The zero field is a solution of eq. (2): every level, max|u| and the
    energy stay exactly 0, and an energy alarm (reference E = 0) never trips."""
    n, steps = 24, 20
    u0 = np.zeros((n, n, n), np.complex128 if complex_field else np.float64)
    with kg.Solver(n, 0.01, precision=precision, complex_field=complex_field,
                   blowup_threshold=1e3) as s:
        s.energy_alarm(1e-12)
        s.set_state(u0)
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        assert not np.any(s.spectrum(0)) and not np.any(s.spectrum(1))
        assert not np.any(s.u())
        assert np.all(s.energies(0, steps + 1) == 0.0)
        elin, q4, maxu = s.records(0, steps)
        assert not np.any(elin) and not np.any(q4) and not np.any(maxu)


def test_zero_amplitude_run_in_a_sweep(kg):
    res, _ = kg.kg_batch_run([dict(n=32, A=0.0, sigma=(1, 1, 1), dt=0.01, max_steps=15,
                                   threshold=1e3),
                              dict(n=48, A=0.0, sigma=(1, 2, 1), dt=0.01, max_steps=0,
                                   threshold=1e3)])
    for r, m in zip(res, (15, 0)):
        assert not r["blew_up"] and r["steps_done"] == m
        assert r["E0"] == 0.0 and r["E_final"] == 0.0 and r["max_abs_u"] == 0.0


@pytest.mark.parametrize("n,precision", [(32, 0), (24, 0), (32, 1)])
def test_other_box_length_matches_oracle(kg, n, precision):
    """A box of side 10 instead of 8 pi (the wavenumbers, h^3 and the sampled
    grid all change): the nonlinear Gaussian after 30 steps against the
    oracle, FP64 to 1e-11 and FP32 to 1e-4, energies alike."""
    Lb, dt, steps = 10.0, 0.01, 30
    u0 = ki.gaussian(n, 1.2, (0.9, 1.1, 1.3), L=Lb)
    ref = oracle.run(u0, dt, steps, L=(Lb,) * 3)
    tol = 1e-11 if precision == 0 else 1e-4
    with kg.Solver(n, dt, L=Lb, precision=precision) as s:
        s.set_state(u0)
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        assert rel_l2(s.u(), ref["u"]) <= tol
        E = s.energies(0, steps + 1)
        assert np.max(np.abs(E - ref["energy"]) / np.abs(ref["energy"])) <= tol


def test_other_box_length_in_a_sweep(kg):
    Lb = 10.0
    runs = [dict(n=32, A=1.2, sigma=(0.9, 1.1, 1.3), dt=0.01, max_steps=30, threshold=1e3),
            dict(n=48, A=4.0, sigma=(1.0, 1.2, 0.9), dt=0.01, max_steps=300, threshold=1e3)]
    res, _ = kg.kg_batch_run(runs, L=Lb)
    for r, b in zip(runs, res):
        ref = oracle.run(ki.gaussian(r["n"], r["A"], r["sigma"], L=Lb), r["dt"], r["max_steps"],
                         L=(Lb,) * 3, threshold=r["threshold"])
        assert b["blew_up"] == (ref["blowup_step"] >= 0)
        assert abs(b["E0"] - ref["energy"][0]) <= 1e-11 * abs(ref["energy"][0])
        if b["blew_up"]:
            assert b["steps_done"] == ref["blowup_step"]
        else:
            E = ref["energy"][r["max_steps"]]
            assert abs(b["E_final"] - E) <= 1e-11 * abs(E)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_time_step_linear(kg, precision):
    """dt = 0.5 (a_k = omega_k^2 dt^2 / 4 from 0.06 to 3.1, so alpha_k runs
    from 1.76 down to -1.0): the semi-implicit scheme of eq. (2) keeps the
    linear energy of Sec. 1.1 exactly for any dt, and the GPU follows the
    oracle (FP64 1e-11; FP32 1e-4, its energy to 1e-6)."""
    n, dt, steps = 32, 0.5, 40
    u0 = ki.gaussian(n, 0.7, (1.3, 0.8, 1.0))
    ref = oracle.run(u0, dt, steps, linear_only=True)
    E_ref = ref["energy"]
    assert np.max(np.abs(E_ref - E_ref[0])) <= 1e-12 * abs(E_ref[0])
    tol, etol = (1e-11, 1e-12) if precision == 0 else (1e-4, 1e-6)
    with kg.Solver(n, dt, linear_only=True, precision=precision) as s:
        s.set_state(u0)
        st, done = s.step(steps)
        assert st == kg.KG_OK and done == steps
        assert rel_l2(s.u(), ref["u"]) <= tol
        E = s.energies(0, steps + 1)
        assert np.max(np.abs(E - E[0])) <= etol * abs(E[0])
        assert np.max(np.abs(E - E_ref)) <= max(etol, 1e-11) * abs(E_ref[0])


def test_library_owned_workspace_matches_borrowed(kg):
    """kg_plan with no workspace allocates and owns its own; the run is
    bitwise the run in a caller's workspace."""
    n, dt, steps = 32, 0.01, 25
    u0 = ki.gaussian(n, 1.2)
    plan = kg.kg_plan(kg.make_params(n, dt))
    try:
        kg.kg_set_state(plan, u0)
        st, done = kg.kg_step(plan, steps, kg.KG_STEP_SYNC)
        assert st == kg.KG_OK and done == steps
        E = kg.kg_energies(plan, 0, steps + 1)
        spec = kg.kg_get_spectrum(plan, n, 0)
    finally:
        kg.kg_destroy(plan)
    with kg.Solver(n, dt) as s:
        s.set_state(u0)
        s.step(steps)
        assert np.array_equal(spec, s.spectrum(0))
        assert np.array_equal(E, s.energies(0, steps + 1))


def test_asynchronous_steps_match_synchronous(kg):
    """kg_step without KG_STEP_SYNC only enqueues graph replays (the path the
    benchmark times): several such calls in a row, then a synchronising
    query, give bitwise the levels and energies of one synchronous call; past
    a blow-up the queued replays do nothing and the counter stays at the
    blown level (the uniform a = 1.5 data blows up at level 145, dt = 0.01)."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.2)
    with kg.Solver(n, dt) as a, kg.Solver(n, dt) as b:
        a.set_state(u0)
        for k in (7, 1, 8, 19):
            st, _ = a.step(k, sync=False)
            assert st == kg.KG_OK
        b.set_state(u0)
        st, done = b.step(35)
        assert st == kg.KG_OK and done == 35
        assert a.stats() == b.stats() == (35, 0, -1)
        assert np.array_equal(a.spectrum(0), b.spectrum(0))
        assert np.array_equal(a.spectrum(1), b.spectrum(1))
        assert np.array_equal(a.energies(0, 36), b.energies(0, 36))
    with kg.Solver(8, dt, blowup_threshold=1e3) as s:
        s.set_state(ki.uniform(8, 1.5))
        for _ in range(20):
            s.step(9, sync=False)  # 180 steps queued, the run blows up at 145
        assert s.stats() == (145, 1, 145)
        st, done = s.step(1)
        assert st == kg.KG_BLOWUP and done == 145
