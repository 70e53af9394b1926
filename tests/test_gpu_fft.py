"""Parity of the solver's transform kernels (through the C-ABI) with the
oracle's FFT: every pass on its own and the full 3D r2c / c2r chains.

Tolerance: the kernels and the oracle both compute O(log n)-deep sums of
rounded products, so they agree to a few units of 1e-16 times log2(n) of the
largest magnitude; 1e-13 leaves a wide margin while any indexing, twiddle or
sign mistake gives errors of order 1.
"""
import numpy as np
import pytest

import kg_inputs as ki
import oracle

pytestmark = pytest.mark.gpu

SIZES = [8, 16, 24, 32, 48, 64, 96, 128, 256]
TOL = 1e-13


def half(n):
    return n // 2 + 1


@pytest.fixture(scope="module")
def plans(kg):
    out = {}
    yield lambda n: out.setdefault(n, kg.Solver(n, 0.01))
    for s in out.values():
        s.close()


@pytest.mark.parametrize("n", SIZES)
def test_forward_r2c_3d(kg, plans, n):
    s = plans(n)
    u = ki.random_field(n, seed=n)
    got = kg.kg_debug_forward(s.plan, u)
    ref = oracle.fft3d(u)[:, :, :half(n)]
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("n", SIZES)
def test_inverse_c2r_3d(kg, plans, n):
    s = plans(n)
    u = ki.random_field(n, seed=100 + n)
    spec = oracle.fft3d(u)[:, :, :half(n)]
    got = kg.kg_debug_inverse(s.plan, spec)
    ref = u * n ** 3  # unnormalised inverse of the forward transform
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("n", SIZES)
def test_c2r_takes_the_real_part(kg, plans, n):
    """A non-Hermitian half spectrum: the c2r result must equal the real part
    of the inverse of its Hermitian completion, i.e. Re of the full inverse
    with the kx > n/2 half filled in by conjugate symmetry."""
    s = plans(n)
    rng = np.random.default_rng(n)
    spec = rng.standard_normal((n, n, half(n))) + 1j * rng.standard_normal((n, n, half(n)))
    full = np.zeros((n, n, n), np.complex128)
    full[:, :, :half(n)] = spec
    # Hermitian completion: X[kz, ky, kx] = conj X[-kz, -ky, -kx] for kx > n/2
    kx = np.arange(half(n), n)
    full[:, :, kx] = np.conj(spec[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, n - kx])
    # planes kx = 0 and n/2 keep only their Hermitian parts
    for k in (0, n // 2):
        p = full[:, :, k]
        full[:, :, k] = 0.5 * (p + np.conj(p[(-np.arange(n)) % n][:, (-np.arange(n)) % n]))
    ref = oracle.fft3d(full, 1).real
    got = kg.kg_debug_inverse(s.plan, spec)
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("which,axis,sign", [(1, 1, -1), (2, 1, 1), (3, 2, -1), (4, 2, 1)])
def test_single_pass(kg, plans, n, which, axis, sign):
    s = plans(n)
    rng = np.random.default_rng(7 * n + which)
    spec = rng.standard_normal((n, n, half(n))) + 1j * rng.standard_normal((n, n, half(n)))
    got = kg.kg_debug_pass(s.plan, which, spec)
    ref = oracle.fft3d_axis(spec, axis, sign)
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


def test_forward_512_sampled(kg):
    """Full size: the 512^3 forward transform at sampled modes against direct sums."""
    n = 512
    with kg.Solver(n, 0.005) as s:
        u = ki.gaussian(n, 0.1, (0.9, 1.1, 1.3), center=(0.3, -0.2, 0.5))
        got = kg.kg_debug_forward(s.plan, u)
    modes = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 5, 7), (256, 0, 0),
             (17, 300, 41), (255, 511, 256), (100, 100, 100)]
    v0, _ = oracle.first_step_modes(u, 0.005, modes)
    scale = np.abs(v0).max()
    for (ix, iy, iz), ref in zip(modes, v0):
        assert abs(got[iz, iy, ix] - ref) <= TOL * scale
