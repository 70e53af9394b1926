"""The energy alarm through the C-ABI (Sec. 1.1: the conserved energy is the
check that code, libraries and hardware computed a run correctly).

Each step compares its E^{n-1/2} with the initial pair's E^{-1/2} on the
device and stops the run at the first level whose relative drift exceeds the
tolerance.  The decision is checked against the energy series the library
reports (kg_energies) for the same run with the alarm off: the run must stop
exactly at the first level where that series drifts past the tolerance, with
records bitwise equal to it up to there.  The fault is forced from the host
by scaling one stored spectral coefficient (kg_debug_scale_mode); every
kernel still runs to completion.
"""
import numpy as np
import pytest

import kg_inputs as ki

pytestmark = pytest.mark.gpu

# (name, n, dt, A, linear_only, precision, fault level, mode (kx, ky, kz), factor)
CASES = [
    ("linear_fp64", 32, 0.01, 0.5, True, 0, 40, (1, 2, 3), 1.001),
    ("nonlinear_fp64", 32, 0.01, 1.5, False, 0, 30, (2, 1, 0), 1.05),
    ("nonlinear_fp32", 32, 0.01, 1.5, False, 1, 30, (2, 1, 0), 1.05),
    ("radix3_fp64", 48, 0.005, 1.0, False, 0, 25, (0, 5, 47), 0.9),
]
STEPS = 60


def first_trip(E, tol):
    """First level m >= 1 whose E^{m-1/2} (E[m]) drifts from E[0] by more
    than tol relative, or -1."""
    bad = ~(np.abs(E[1:] - E[0]) <= tol * abs(E[0]))
    idx = np.nonzero(bad)[0]
    return int(idx[0]) + 1 if idx.size else -1


def faulted_run(kg, case, tol):
    """The case's run with the fault at its level; tol = None: alarm off."""
    _, n, dt, A, lin, prec, at, mode, factor = case
    with kg.Solver(n, dt, linear_only=lin, precision=prec) as s:
        if tol is not None:
            s.energy_alarm(tol)
        s.set_state(ki.gaussian(n, A, (1.0, 0.8, 1.2)))
        st, done = s.step(at)
        assert st == kg.KG_OK and done == at
        assert kg.kg_debug_scale_mode(s.plan, *mode, factor) == kg.KG_OK
        st, done = s.step(STEPS - at)
        stats = s.stats()
        top = stats[0]
        # a stopped run has the record of its stopping level; a running one
        # records a level when it steps from it
        recs = s.records(0, top + 1 if stats[1] else top)
        E = s.energies(0, top + 1)
        spec1_ok = True
        if stats[1]:
            with pytest.raises(kg.KGError) as e:
                s.spectrum(1)
            spec1_ok = e.value.status == kg.KG_E_INVALID
            assert np.isnan(s.energy()[0])
        return st, done, stats, recs, E, spec1_ok


def natural_drift(kg, case):
    """Largest relative energy drift of the case's run without the fault."""
    _, n, dt, A, lin, prec, _, _, _ = case
    with kg.Solver(n, dt, linear_only=lin, precision=prec) as s:
        s.set_state(ki.gaussian(n, A, (1.0, 0.8, 1.2)))
        s.step(STEPS)
        E = s.energies(0, STEPS + 1)
    return float(np.max(np.abs(E - E[0])) / abs(E[0]))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_alarm_stops_where_the_energy_series_drifts(kg, case):
    drift = natural_drift(kg, case)
    tol = 1e-11 if case[4] else 4.0 * drift
    assert drift < tol
    # the same faulted run without the alarm: where its energy series trips
    st, done, stats, (elin, q4, maxu), E, _ = faulted_run(kg, case, None)
    assert st == kg.KG_OK and done == STEPS and stats[1] == 0
    trip = first_trip(E, tol)
    at = case[6]
    assert at <= trip <= at + 1, (trip, at)  # nothing before the fault, then at once
    # with the alarm: stops there, records equal up to it
    st, done, stats, (elin_a, q4_a, maxu_a), E_a, spec1_ok = faulted_run(kg, case, tol)
    assert st == kg.KG_E_ENERGY and done == trip
    assert stats == (trip, 2, trip)
    assert np.array_equal(elin_a, elin[:trip + 1]) and np.array_equal(q4_a, q4[:trip + 1])
    assert np.array_equal(maxu_a, maxu[:trip + 1])
    assert np.array_equal(E_a, E[:trip + 1])
    assert spec1_ok  # the stopping step has overwritten v^{n-1}, as on a blow-up


def test_alarm_changes_nothing_until_it_trips(kg):
    """A run with the alarm set above its drift is bitwise the run without it."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 1.5)
    out = []
    for tol in (None, 0.5):
        with kg.Solver(n, dt) as s:
            if tol is not None:
                s.energy_alarm(tol)
            s.set_state(u0)
            st, done = s.step(50)
            assert st == kg.KG_OK and done == 50
            out.append((s.spectrum(0), s.spectrum(1), s.energies(0, 51)))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_alarm_setting_and_reference_survive_state_calls(kg):
    """The tolerance belongs to the plan (kept across kg_set_state and
    kg_load_state); the reference energy belongs to the run (saved with it)."""
    n, dt = 32, 0.01
    u0 = ki.gaussian(n, 0.5)
    with kg.Solver(n, dt, linear_only=True) as s, kg.Solver(n, dt, linear_only=True) as t:
        s.energy_alarm(1e-11)        # set before the state
        s.set_state(u0)
        st, done = s.step(20)
        assert st == kg.KG_OK and done == 20
        buf = s.save()
        # reload into the same plan: no false alarm (reference kept), then a fault trips it
        s.load(buf)
        st, done = s.step(20)
        assert st == kg.KG_OK and done == 40
        kg.kg_debug_scale_mode(s.plan, 1, 0, 0, 1.01)
        st, done = s.step(5)
        assert st == kg.KG_E_ENERGY and done == 41
        # a plan without the alarm runs the same faulted state on
        t.load(buf)
        kg.kg_debug_scale_mode(t.plan, 1, 0, 0, 1.01)
        st, done = t.step(5)
        assert st == kg.KG_OK and done == 25
        # a new state keeps the plan's setting
        s.set_state(u0)
        st, done = s.step(3)
        assert st == kg.KG_OK and done == 3
        kg.kg_debug_scale_mode(s.plan, 0, 1, 0, 1.01)
        st, done = s.step(3)
        assert st == kg.KG_E_ENERGY and done == 4
        # 0 turns it off
        s.set_state(u0)
        s.energy_alarm(0.0)
        s.step(3)
        kg.kg_debug_scale_mode(s.plan, 0, 1, 0, 1.01)
        st, done = s.step(3)
        assert st == kg.KG_OK and done == 6


@pytest.mark.parametrize("precision,complex_field", [(0, False), (1, False), (0, True),
                                                     (1, True)])
def test_scale_mode_changes_one_coefficient(kg, precision, complex_field):
    """The forced fault multiplies exactly one stored coefficient of v^n and
    leaves v^{n-1} as it was (complex fields: the full spectrum, kx up to n)."""
    n, dt = 24, 0.01
    kx, ky, kz, f = (19 if complex_field else 3), 5, 20, 1.25
    with kg.Solver(n, dt, precision=precision, complex_field=complex_field) as s:
        u0 = ki.gaussian(n, 1.0)
        s.set_state(u0 * np.exp(0.5j * ki.axis(n)) if complex_field else u0)
        s.step(7)
        v0, w0 = s.spectrum(0), s.spectrum(1)
        assert kg.kg_debug_scale_mode(s.plan, kx, ky, kz, f) == kg.KG_OK
        v1, w1 = s.spectrum(0), s.spectrum(1)
    mask = np.zeros(v0.shape, bool)
    mask[kz, ky, kx] = True
    assert np.array_equal(v1[~mask], v0[~mask])
    if precision == 0:
        assert v1[kz, ky, kx] == f * v0[kz, ky, kx]
        assert np.array_equal(w1, w0)
    else:  # float storage of v and its increment
        assert abs(v1[kz, ky, kx] - f * v0[kz, ky, kx]) <= 2e-7 * abs(v0[kz, ky, kx])
        assert np.array_equal(w1[~mask], w0[~mask])
        assert abs(w1[kz, ky, kx] - w0[kz, ky, kx]) <= 1e-6 * abs(v0[kz, ky, kx])


def test_alarm_and_scale_mode_argument_checks(kg):
    with kg.Solver(16, 0.01) as s:
        for bad in (-1e-3, float("nan"), float("inf")):
            with pytest.raises(kg.KGError) as e:
                s.energy_alarm(bad)
            assert e.value.status == kg.KG_E_INVALID
        with pytest.raises(kg.KGError) as e:  # before any state
            kg.kg_debug_scale_mode(s.plan, 0, 0, 0, 2.0)
        assert e.value.status == kg.KG_E_INVALID
        s.set_state(ki.gaussian(16, 0.5))
        for args in ((9, 0, 0, 2.0), (0, 16, 0, 2.0), (0, 0, -1, 2.0), (0, 0, 0, float("inf"))):
            with pytest.raises(kg.KGError) as e:
                kg.kg_debug_scale_mode(s.plan, *args)
            assert e.value.status == kg.KG_E_INVALID
