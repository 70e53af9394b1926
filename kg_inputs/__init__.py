"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Holds none of the solver's arithmetic: only grids, initial fields sampled from
closed-form functions, and parameter draws.  Fields are float64 arrays in
[z][y][x] order (x fastest) on the periodic box [-L/2, L/2)^3 with grid points
x_j = -L/2 + j*h, h = L/n.
"""
import numpy as np

BOX = 8.0 * np.pi  # [-4 pi, 4 pi) per axis


def axis(n, L=BOX):
    """Grid coordinates x_j = -L/2 + j L/n, j = 0..n-1."""
    return -0.5 * L + (L / n) * np.arange(n, dtype=np.float64)


def mesh(n, L=BOX):
    """Broadcastable (z, y, x) coordinate arrays for an n^3 grid (n may be a 3-tuple
    (nx, ny, nz) and L a 3-tuple (Lx, Ly, Lz))."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    Lx, Ly, Lz = (L, L, L) if np.isscalar(L) else L
    x = axis(nx, Lx)[None, None, :]
    y = axis(ny, Ly)[None, :, None]
    z = axis(nz, Lz)[:, None, None]
    return z, y, x


def gaussian(n, A=0.1, sigma=(1.0, 1.0, 1.0), L=BOX, center=(0.0, 0.0, 0.0)):
    """u0 = A exp(-((x-cx)^2/sx^2 + (y-cy)^2/sy^2 + (z-cz)^2/sz^2)); sigma = (sx, sy, sz),
    center = (cx, cy, cz)."""
    z, y, x = mesh(n, L)
    sx, sy, sz = sigma
    x, y, z = x - center[0], y - center[1], z - center[2]
    return np.ascontiguousarray(A * np.exp(-(x * x / (sx * sx) + y * y / (sy * sy) +
                                            z * z / (sz * sz))))


def plane_wave(n, mode, phase=0.0, L=BOX, fn=np.cos):
    """fn(k.x + phase) with k = 2 pi mode / L (mode = integer (mx, my, mz))."""
    z, y, x = mesh(n, L)
    Lx, Ly, Lz = (L, L, L) if np.isscalar(L) else L
    kx, ky, kz = (2 * np.pi * mode[0] / Lx, 2 * np.pi * mode[1] / Ly, 2 * np.pi * mode[2] / Lz)
    return np.ascontiguousarray(fn(kx * x + ky * y + kz * z + phase) + 0.0 * (x + y + z))


def uniform(n, a):
    """Spatially constant field of value a."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return np.full((nz, ny, nx), float(a))


def random_field(n, seed, scale=1.0):
    """Seeded standard-normal field (for transform tests)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return scale * np.random.default_rng(seed).standard_normal((nz, ny, nx))


SWEEP_SIZES = (48, 64, 96, 128)


def sweep_runs(nruns=512, seed=0, sizes=SWEEP_SIZES):
    """Parametric blow-up sweep: per run, in this order, N uniform over `sizes`,
    A ~ U[0.5, 4], then sx, sy, sz ~ U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    runs = []
    for _ in range(nruns):
        n = int(rng.choice(sizes))
        A = float(rng.uniform(0.5, 4.0))
        s = rng.uniform(0.5, 2.0, size=3)
        runs.append(dict(n=n, A=A, sigma=(float(s[0]), float(s[1]), float(s[2]))))
    return runs


def surrogate_params(nruns, seed):
    """(A, sx, sy, sz) draws of the sweep distribution at a fixed grid size."""
    rng = np.random.default_rng(seed)
    out = np.empty((nruns, 4))
    for i in range(nruns):
        out[i, 0] = rng.uniform(0.5, 4.0)
        out[i, 1:] = rng.uniform(0.5, 2.0, size=3)
    return out
