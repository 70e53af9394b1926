"""Pins for the oracle's FFT against brute-force DFTs and exact transforms.

The paper's method needs two 3D FFTs per step (Sec. 1.1.2, closing paragraph);
the oracle carries its own mixed-radix transform.  Here it is checked against
the DFT definition summed directly, against exactly known transforms, and
against an independent library FFT.
"""
import numpy as np
import pytest

import oracle


def dft_matrix(n, sign=-1):
    j = np.arange(n)
    # exponent reduced mod n in integers so the phases are exact
    return np.exp(sign * 2j * np.pi * ((np.outer(j, j)) % n) / n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 18, 27, 48, 64, 96, 128])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_vs_direct_dft(n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n, sign) @ x
    got = oracle.fft1d(x, sign)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def brute_force_dft3(x, sign=-1):
    """X[k] = sum_j x[j] exp(sign 2 pi i (kx jx/nx + ky jy/ny + kz jz/nz)), O(M^2)."""
    nz, ny, nx = x.shape
    jz, jy, jx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    jz, jy, jx = jz.ravel(), jy.ravel(), jx.ravel()
    xf = x.ravel()
    out = np.empty(xf.size, np.complex128)
    blk = 512
    for s in range(0, xf.size, blk):
        kz, ky, kx = jz[s:s + blk, None], jy[s:s + blk, None], jx[s:s + blk, None]
        ph = ((kx * jx[None, :]) % nx) / nx + ((ky * jy[None, :]) % ny) / ny + \
             ((kz * jz[None, :]) % nz) / nz
        out[s:s + blk] = np.exp(sign * 2j * np.pi * ph) @ xf
    return out.reshape(x.shape)


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 16, 16), (6, 4, 8)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft3d_vs_brute_force(shape, sign):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_force_dft3(x, sign)
    got = oracle.fft3d(x, sign)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fft_axis_is_the_named_axis(axis):
    """Anisotropic shape: a transform along the wrong axis cannot match."""
    rng = np.random.default_rng(axis)
    x = rng.standard_normal((6, 8, 12)) + 1j * rng.standard_normal((6, 8, 12))
    np_axis = 2 - axis  # numpy axes of a [z][y][x] array
    ref = np.apply_along_axis(lambda v: dft_matrix(v.size) @ v, np_axis, x)
    got = oracle.fft3d_axis(x, axis)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fft3d_vs_library_fft():
    """Independent implementation cross-check on a larger, ragged-radix grid."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal((24, 48, 32)) + 1j * rng.standard_normal((24, 48, 32))
    ref = np.fft.fftn(x)
    assert np.abs(oracle.fft3d(x) - ref).max() <= 1e-13 * np.abs(ref).max()
    refi = np.fft.ifftn(x) * x.size
    assert np.abs(oracle.fft3d(x, 1) - refi).max() <= 1e-13 * np.abs(refi).max()


def test_round_trip_and_parseval():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((32, 32, 32))
    X = oracle.fft3d(x)
    back = oracle.fft3d(X, 1) / x.size
    assert np.abs(back - x).max() <= 1e-14 * np.abs(x).max() * 10
    # Parseval: sum |x|^2 = (1/M) sum |X|^2
    assert abs(np.sum(x * x) - np.sum(np.abs(X) ** 2) / x.size) <= 1e-12 * np.sum(x * x)


def test_delta_and_cosine():
    n = 16
    d = np.zeros((n, n, n))
    d[0, 0, 0] = 1.0
    assert np.abs(oracle.fft3d(d) - 1.0).max() <= 1e-15
    # a single cosine cos(2 pi m x_j / n) has two spikes of height M/2 at +-m
    j = np.arange(n)
    m = 3
    c = np.cos(2 * np.pi * m * j / n)[None, None, :] * np.ones((n, n, 1))
    C = oracle.fft3d(c)
    expect = np.zeros((n, n, n), np.complex128)
    expect[0, 0, m] = expect[0, 0, n - m] = n ** 3 / 2
    assert np.abs(C - expect).max() <= 1e-10
