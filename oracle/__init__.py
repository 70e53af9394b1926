"""CPU oracle for the Klein-Gordon spectral solver -- TEST INFRASTRUCTURE.

A plain, slow, double-precision reference written from the paper (the cubic
Klein-Gordon equation of Sec. 1, eq. (1), real fields; the second-order
semi-implicit scheme of Sec. 1.1.2, eq. (2); the energy of Sec. 1.1), with its
own FFT.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  It shares no code with the GPU
library and never imports it.

All arrays are numpy float64 (real fields) or complex128 (spectra) in
[z][y][x] order, x fastest.  Transforms are unnormalised, forward sign -1.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

INIT_VELOCITY = 0
INIT_TWO_LEVEL = 1

class Oracle:
    """The oracle's entry points bound to one compiled library."""

    def __init__(self, path=LIB):
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.kgo_fft1d.argtypes = [ctypes.c_int, dp, ctypes.c_int]
        lib.kgo_fft3d.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int]
        lib.kgo_fft3d_axis.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int, ctypes.c_int]
        lib.kgo_run.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 4 +
                                [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp,
                                 ctypes.c_int, dp, dp, dp, dp, dp, ip, dp])
        lib.kgo_state.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 4 +
                                  [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                   dp, dp])
        lib.kgo_first_step_modes.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 4 +
                                             [ctypes.c_int, dp, ctypes.c_int, ip, dp, dp])
        lib.kgo_run_c.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 4 +
                                  [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp,
                                   ctypes.c_int, dp, dp, dp, dp, dp, ip])
        lib.kgo_num_threads.argtypes = []
        for f in (lib.kgo_fft1d, lib.kgo_fft3d, lib.kgo_fft3d_axis, lib.kgo_run, lib.kgo_state,
                  lib.kgo_first_step_modes, lib.kgo_num_threads, lib.kgo_run_c):
            f.restype = ctypes.c_int
        self.lib = lib

    def num_threads(self):
        """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
        return self.lib.kgo_num_threads()

    def fft1d(self, x, sign=-1):
        """Unnormalised DFT of a 1D complex array (sign -1 forward, +1 inverse)."""
        a = np.ascontiguousarray(x, dtype=np.complex128).copy()
        _check(self.lib.kgo_fft1d(a.size, _ptr(a.view(np.float64)), sign), "fft1d")
        return a

    def fft3d(self, x, sign=-1):
        """Unnormalised 3D DFT of a [z][y][x] array."""
        a = np.ascontiguousarray(x, dtype=np.complex128).copy()
        nz, ny, nx = a.shape
        _check(self.lib.kgo_fft3d(nx, ny, nz, _ptr(a.view(np.float64)), sign), "fft3d")
        return a

    def fft3d_axis(self, x, axis, sign=-1):
        """Unnormalised DFT along one axis (0 = x, 1 = y, 2 = z) of a [z][y][x] array."""
        a = np.ascontiguousarray(x, dtype=np.complex128).copy()
        nz, ny, nx = a.shape
        _check(self.lib.kgo_fft3d_axis(nx, ny, nz, _ptr(a.view(np.float64)), axis, sign),
               "fft3d_axis")
        return a

    def run(self, u0, dt, nsteps, L=(8 * np.pi,) * 3, linear_only=False, threshold=0.0,
            mode=INIT_VELOCITY, aux=None, dealias=False):
        """Step eq. (2) ``nsteps`` times from ``u0`` (and ``aux`` = u_t(0) or u^{-1}).
        ``dealias`` truncates the nonlinear term by the 2/3 rule.

        Returns a dict with ``u`` (u^nsteps or the blown-up level), ``u_prev``,
        ``energy`` (E^{-1/2}, E^{1/2}, ...), ``maxu`` and ``q4`` per level,
        ``blowup_step`` (-1 if none) and ``loop_seconds`` (wall time of the
        steps without set-up).  ``L`` is (Lx, Ly, Lz).
        """
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        nz, ny, nx = u0.shape
        if aux is not None:
            aux = np.ascontiguousarray(aux, dtype=np.float64)
            assert aux.shape == u0.shape
        u = np.empty_like(u0)
        up = np.empty_like(u0)
        energy = np.empty(nsteps + 1)
        maxu = np.empty(nsteps + 1)
        q4 = np.empty(nsteps + 1)
        blow = ctypes.c_int(-1)
        secs = ctypes.c_double(0.0)
        _check(self.lib.kgo_run(nx, ny, nz, L[0], L[1], L[2], dt, int(bool(linear_only)),
                                int(bool(dealias)), float(threshold), mode, _ptr(u0), _ptr(aux), nsteps, _ptr(u),
                                _ptr(up), _ptr(energy), _ptr(maxu), _ptr(q4),
                                ctypes.byref(blow), ctypes.byref(secs)), "run")
        return dict(u=u, u_prev=up, energy=energy, maxu=maxu, q4=q4, blowup_step=blow.value,
                    loop_seconds=secs.value)

    def run_complex(self, u0, dt, nsteps, L=(8 * np.pi,) * 3, linear_only=False, threshold=0.0,
                    mode=INIT_VELOCITY, aux=None, dealias=False):
        """``run`` for a complex field (nonlinear term |u|^2 u): ``u0``, ``aux``
        and the returned ``u``, ``u_prev`` are complex; ``maxu`` = max|u|,
        ``q4`` = h^3 sum |u|^4."""
        u0 = np.ascontiguousarray(u0, dtype=np.complex128)
        nz, ny, nx = u0.shape
        if aux is not None:
            aux = np.ascontiguousarray(aux, dtype=np.complex128)
            assert aux.shape == u0.shape
        u = np.empty_like(u0)
        up = np.empty_like(u0)
        energy = np.empty(nsteps + 1)
        maxu = np.empty(nsteps + 1)
        q4 = np.empty(nsteps + 1)
        blow = ctypes.c_int(-1)
        _check(self.lib.kgo_run_c(nx, ny, nz, L[0], L[1], L[2], dt, int(bool(linear_only)),
                                  int(bool(dealias)), float(threshold), mode, _ptr(u0.view(np.float64)),
                                  _ptr(None if aux is None else aux.view(np.float64)), nsteps,
                                  _ptr(u.view(np.float64)), _ptr(up.view(np.float64)),
                                  _ptr(energy), _ptr(maxu), _ptr(q4), ctypes.byref(blow)),
               "run_complex")
        return dict(u=u, u_prev=up, energy=energy, maxu=maxu, q4=q4, blowup_step=blow.value)

    def state(self, u0, dt, nsteps, L=(8 * np.pi,) * 3, linear_only=False, mode=INIT_VELOCITY,
              aux=None, dealias=False):
        """Full complex spectra (v^{nsteps-1}, v^nsteps) after ``nsteps`` steps."""
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        nz, ny, nx = u0.shape
        if aux is not None:
            aux = np.ascontiguousarray(aux, dtype=np.float64)
        vp = np.empty(u0.shape, np.complex128)
        vc = np.empty(u0.shape, np.complex128)
        _check(self.lib.kgo_state(nx, ny, nz, L[0], L[1], L[2], dt, int(bool(linear_only)),
                                  int(bool(dealias)), mode, _ptr(u0), _ptr(aux), nsteps, _ptr(vp.view(np.float64)),
                                  _ptr(vc.view(np.float64))), "state")
        return vp, vc


    def first_step_modes(self, u0, dt, modes, L=(8 * np.pi,) * 3, linear_only=False):
        """(v^0, v^1) at the given mode index triples (ix, iy, iz), u_t(0) = 0,
        each by direct summation of the DFT definition."""
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        nz, ny, nx = u0.shape
        m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32).reshape(-1, 3))
        v0 = np.empty(len(m), np.complex128)
        v1 = np.empty(len(m), np.complex128)
        _check(self.lib.kgo_first_step_modes(
            nx, ny, nz, L[0], L[1], L[2], dt, int(bool(linear_only)), _ptr(u0), len(m),
            m.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(v0.view(np.float64)),
            _ptr(v1.view(np.float64))), "first_step_modes")
        return v0, v1


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


_default = None


def default():
    """The oracle built from this directory (compiled on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build_oracle()
        _default = Oracle(LIB)
    return _default


def num_threads():
    return default().num_threads()


def fft1d(x, sign=-1):
    return default().fft1d(x, sign)


def fft3d(x, sign=-1):
    return default().fft3d(x, sign)


def fft3d_axis(x, axis, sign=-1):
    return default().fft3d_axis(x, axis, sign)


def run(*args, **kw):
    return default().run(*args, **kw)


def run_complex(*args, **kw):
    return default().run_complex(*args, **kw)


def state(*args, **kw):
    return default().state(*args, **kw)


def first_step_modes(*args, **kw):
    return default().first_step_modes(*args, **kw)
