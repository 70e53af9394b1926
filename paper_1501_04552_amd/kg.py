"""ctypes binding of libkg.so, the HIP (gfx950) Klein-Gordon spectral stepper.

The functions keep the C names of ``include/kg.h`` and only marshal
arguments; every step of the solver runs in the library's kernels.  PyTorch
supplies device memory (the workspace, device-resident fields) and the HIP
stream.  Importing fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (load PyTorch's HIP runtime before the library)

from .build import LIB

if not os.path.exists(LIB):
    raise ImportError(f"{LIB} is missing: build it with `python paper_1501_04552_amd/build.py` "
                      "or __graft_entry__.build()")

_lib = ctypes.CDLL(LIB)

KG_OK, KG_E_INVALID, KG_E_UNSUPPORTED_SIZE, KG_E_NOMEM, KG_E_HIP, KG_BLOWUP, KG_E_ENERGY = range(7)
KG_FP64, KG_FP32 = 0, 1
KG_INIT_VELOCITY, KG_INIT_TWO_LEVEL = 0, 1
KG_STEP_SYNC = 1
KG_STEP_TIMED = 2

# names of the step kernels for kg_debug_time_kernel / kg_kernel_bytes
KERNELS = ("x_pass", "y_forward", "z_update", "y_inverse", "finalize")


class kg_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int), ("linear_only", ctypes.c_int),
                ("blowup_threshold", ctypes.c_double), ("complex_field", ctypes.c_int),
                ("dealias", ctypes.c_int)]


class kg_run_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("A", ctypes.c_double), ("sx", ctypes.c_double),
                ("sy", ctypes.c_double), ("sz", ctypes.c_double), ("dt", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("threshold", ctypes.c_double)]


class kg_run_result(ctypes.Structure):
    _fields_ = [("blew_up", ctypes.c_int), ("steps_done", ctypes.c_int),
                ("t_blowup", ctypes.c_double), ("E0", ctypes.c_double),
                ("E_final", ctypes.c_double), ("max_abs_u", ctypes.c_double)]


class kg_batch_opts(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("graph_steps", ctypes.c_int), ("tune", ctypes.c_int),
                ("tune_cache", ctypes.c_char_p), ("seconds", ctypes.POINTER(ctypes.c_double))]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_pp = ctypes.POINTER(ctypes.c_void_p)
_P = ctypes.POINTER(kg_params)

_SIGS = {
    "kg_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "kg_last_error": (ctypes.c_char_p, [_vp]),
    "kg_workspace_bytes": (ctypes.c_size_t, [_P]),
    "kg_plan": (ctypes.c_int, [_P, _vp, ctypes.c_size_t, _vp, _pp]),
    "kg_destroy": (None, [_vp]),
    "kg_set_state": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    "kg_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint, _ip]),
    "kg_energy": (ctypes.c_int, [_vp, _dp, _dp]),
    "kg_records": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "kg_energies": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp]),
    "kg_stats": (ctypes.c_int, [_vp, _ip, _ip, _ip, _dp]),
    "kg_set_energy_alarm": (ctypes.c_int, [_vp, ctypes.c_double]),
    "kg_get_u": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "kg_get_state": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "kg_get_spectrum": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "kg_state_bytes": (ctypes.c_size_t, [_vp]),
    "kg_save_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "kg_load_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "kg_debug_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "kg_debug_inverse": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "kg_debug_pass": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "kg_debug_time_kernel": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_float)]),
    "kg_debug_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp,
                                     ctypes.POINTER(ctypes.c_float)]),
    "kg_debug_scale_mode": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double]),
    "kg_kernel_bytes": (ctypes.c_double, [_vp, ctypes.c_int]),
    "kg_kernel_times": (ctypes.c_int, [_vp, _dp, _ip]),
    "kg_batch_run": (ctypes.c_int, [ctypes.POINTER(kg_run_desc), ctypes.c_int,
                                    ctypes.POINTER(kg_run_result), ctypes.POINTER(kg_batch_opts),
                                    _vp]),
    "kg_batch_last_error": (ctypes.c_char_p, []),
    "kg_mlp_num_params": (ctypes.c_size_t, [ctypes.c_int]),
    "kg_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, _vp, _pp]),
    "kg_mlp_destroy": (None, [_vp]),
    "kg_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "kg_mlp_set_norm": (ctypes.c_int, [_vp, _vp, _vp]),
    "kg_mlp_get_params": (ctypes.c_int, [_vp, _vp]),
    "kg_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    "kg_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "kg_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp]),
    "kg_mlp_forward_noalloc": (ctypes.c_int, [ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, _vp,
                                              _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_SIGS)


class KGError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{kg_status_str(status)}{': ' + msg if msg else ''}")


def kg_status_str(status):
    return _lib.kg_status_str(status).decode()


def kg_last_error(plan):
    return _lib.kg_last_error(plan).decode()


def _check(status, plan=None, allow=(KG_OK,)):
    if status not in allow:
        raise KGError(status, kg_last_error(plan) if plan else "")
    return status


def make_params(n, dt, L=0.0, precision=KG_FP64, linear_only=False, blowup_threshold=0.0,
                complex_field=False, dealias=False):
    return kg_params(int(n), float(L), float(dt), int(precision), int(bool(linear_only)),
                     float(blowup_threshold), int(bool(complex_field)), int(bool(dealias)))


def kg_workspace_bytes(params):
    return _lib.kg_workspace_bytes(ctypes.byref(params))


def kg_plan(params, workspace_ptr=None, ws_bytes=0, stream=None):
    out = ctypes.c_void_p()
    _check(_lib.kg_plan(ctypes.byref(params), workspace_ptr, ws_bytes, stream, ctypes.byref(out)))
    return out.value


def kg_destroy(plan):
    _lib.kg_destroy(plan)


def _buf(x):
    """(pointer, on_device) of a numpy array or a torch tensor (float64, or
    complex128 for complex fields: interleaved re, im)."""
    if x is None:
        return None, 0
    if isinstance(x, np.ndarray):
        assert x.flags.c_contiguous and x.dtype in (np.float64, np.complex128)
        return x.ctypes.data, 0
    assert x.is_contiguous() and x.is_cuda and x.dtype in (torch.float64, torch.complex128)
    return x.data_ptr(), 1


def kg_set_state(plan, u0, aux=None, mode=KG_INIT_VELOCITY):
    p0, d0 = _buf(u0)
    pa, da = _buf(aux)
    if aux is not None and da != d0:
        raise ValueError("u0 and aux must both be host or both be device arrays")
    _check(_lib.kg_set_state(plan, p0, pa, mode, d0), plan)


def kg_step(plan, nsteps, flags=0):
    done = ctypes.c_int(-1)
    st = _check(_lib.kg_step(plan, nsteps, flags, ctypes.byref(done)), plan,
                allow=(KG_OK, KG_BLOWUP, KG_E_ENERGY))
    return st, done.value


def kg_energy(plan):
    E, t = ctypes.c_double(), ctypes.c_double()
    st = _check(_lib.kg_energy(plan, ctypes.byref(E), ctypes.byref(t)), plan,
                allow=(KG_OK, KG_BLOWUP, KG_E_ENERGY))
    return (E.value, t.value) if st == KG_OK else (float("nan"), float("nan"))


def kg_records(plan, first, count):
    elin, q4, maxu = np.empty(count), np.empty(count), np.empty(count)
    _check(_lib.kg_records(plan, first, count, elin.ctypes.data, q4.ctypes.data,
                           maxu.ctypes.data), plan)
    return elin, q4, maxu


def kg_energies(plan, first, count):
    """E^{m-1/2} for levels m = first .. first+count-1 (host array)."""
    E = np.empty(count)
    _check(_lib.kg_energies(plan, first, count, E.ctypes.data), plan)
    return E


def kg_stats(plan, max_abs_u=False):
    """(steps done, stop flag (0 running, 1 blown up, 2 energy alarm), the
    level the run stopped at or -1), plus max|u^n| of the newest level when
    max_abs_u is true."""
    s, b, bs, mx = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_lib.kg_stats(plan, ctypes.byref(s), ctypes.byref(b), ctypes.byref(bs),
                         ctypes.byref(mx) if max_abs_u else None), plan)
    if max_abs_u:
        return s.value, b.value, bs.value, mx.value
    return s.value, b.value, bs.value


def kg_set_energy_alarm(plan, rel_tol):
    _check(_lib.kg_set_energy_alarm(plan, float(rel_tol)), plan)


def kg_get_u(plan, n, out=None, complex_field=False):
    if out is None:
        out = np.empty((n, n, n), np.complex128 if complex_field else np.float64)
    p, d = _buf(out)
    _check(_lib.kg_get_u(plan, p, d), plan)
    return out


def kg_get_state(plan, n, u_prev=None, u_cur=None, complex_field=False, want_prev=True):
    """(u^{n-1}, u^n) in physical space; outputs are allocated on the host
    when not given (u^{n-1} is None when want_prev is false)."""
    dt = np.complex128 if complex_field else np.float64
    if u_prev is None and want_prev:
        u_prev = np.empty((n, n, n), dt)
    if u_cur is None:
        u_cur = np.empty((n, n, n), dt)
    pp, dp = _buf(u_prev)
    pc, dc = _buf(u_cur)
    if u_prev is not None and dp != dc:
        raise ValueError("u_prev and u_cur must both be host or both be device arrays")
    _check(_lib.kg_get_state(plan, pp, pc, dc), plan)
    return u_prev, u_cur


def kg_get_spectrum(plan, n, which=0, out=None, complex_field=False):
    """Half spectrum [kz][ky][kx<=n/2] of v^n (which=0) or v^{n-1} (which=1);
    the full spectrum [kz][ky][kx] for a complex field."""
    if out is None:
        out = np.empty((n, n, n if complex_field else n // 2 + 1), np.complex128)
    _check(_lib.kg_get_spectrum(plan, which, out.ctypes.data, 0), plan)
    return out


def kg_state_bytes(plan):
    return _lib.kg_state_bytes(plan)


def kg_save_state(plan):
    buf = np.empty(kg_state_bytes(plan), np.uint8)
    _check(_lib.kg_save_state(plan, buf.ctypes.data, buf.size), plan)
    return buf


def kg_load_state(plan, buf):
    buf = np.ascontiguousarray(buf, np.uint8)
    _check(_lib.kg_load_state(plan, buf.ctypes.data, buf.size), plan)


def kg_debug_forward(plan, u):
    n = u.shape[0]
    spec = np.empty((n, n, n if np.iscomplexobj(u) else n // 2 + 1), np.complex128)
    _check(_lib.kg_debug_forward(plan, u.ctypes.data, spec.ctypes.data, 0), plan)
    return spec


def kg_debug_inverse(plan, spec):
    """Inverse 3D transform (with 1/M) of a half spectrum, or of a full one
    (complex field plans: last axis n) into a complex field."""
    n = spec.shape[0]
    spec = np.ascontiguousarray(spec, np.complex128)
    u = np.empty((n, n, n), np.complex128 if spec.shape[2] == n else np.float64)
    _check(_lib.kg_debug_inverse(plan, spec.ctypes.data, u.ctypes.data, 0), plan)
    return u


def kg_debug_pass(plan, which, spec):
    spec = np.ascontiguousarray(spec, np.complex128).copy()
    _check(_lib.kg_debug_pass(plan, which, spec.ctypes.data, 0), plan)
    return spec


def kg_debug_time_kernel(plan, kernel, reps):
    ms = ctypes.c_float()
    _check(_lib.kg_debug_time_kernel(plan, kernel, reps, ctypes.byref(ms)), plan)
    return ms.value


def kg_debug_scale_mode(plan, kx, ky, kz, factor):
    return _check(_lib.kg_debug_scale_mode(plan, kx, ky, kz, float(factor)), plan,
                  allow=(KG_OK, KG_BLOWUP, KG_E_ENERGY))


def kg_debug_copy(dst_ptr, src_ptr, nbytes, reps, stream=None):
    ms = ctypes.c_float()
    _check(_lib.kg_debug_copy(dst_ptr, src_ptr, nbytes, reps, stream, ctypes.byref(ms)))
    return ms.value


def kg_kernel_times(plan):
    """(average ms per kernel [x, y fwd, z, y inv, finalize], steps averaged)."""
    ms = (ctypes.c_double * 5)()
    n = ctypes.c_int()
    _check(_lib.kg_kernel_times(plan, ms, ctypes.byref(n)), plan)
    return list(ms), n.value


def kg_kernel_bytes(plan, kernel):
    return _lib.kg_kernel_bytes(plan, kernel)


def kg_batch_run(runs, L=0.0, graph_steps=0, tune=False, tune_cache=None, stream=None):
    """Run a sweep.  runs: sequence of dicts with n, A, sigma (sx, sy, sz), dt,
    max_steps, threshold.  Returns (list of result dicts, stepping seconds)."""
    nr = len(runs)
    desc = (kg_run_desc * nr)()
    for d, r in zip(desc, runs):
        sx, sy, sz = r["sigma"]
        d.n, d.A, d.sx, d.sy, d.sz = int(r["n"]), float(r["A"]), float(sx), float(sy), float(sz)
        d.dt, d.max_steps, d.threshold = float(r["dt"]), int(r["max_steps"]), float(r["threshold"])
    out = (kg_run_result * nr)()
    secs = ctypes.c_double(0.0)
    opts = kg_batch_opts(float(L), int(graph_steps), int(bool(tune)),
                         tune_cache.encode() if tune_cache else None, ctypes.pointer(secs))
    st = _lib.kg_batch_run(desc, nr, out, ctypes.byref(opts), stream)
    if st != KG_OK:
        raise KGError(st, _lib.kg_batch_last_error().decode())
    res = [dict(blew_up=bool(o.blew_up), steps_done=o.steps_done, t_blowup=o.t_blowup, E0=o.E0,
                E_final=o.E_final, max_abs_u=o.max_abs_u) for o in out]
    return res, secs.value


def _mcheck(status, m):
    if status != KG_OK:
        raise KGError(status, _lib.kg_mlp_last_error(m).decode() if m else "")


def kg_mlp_num_params(hidden):
    return _lib.kg_mlp_num_params(hidden)


def kg_mlp_create(hidden, max_batch, init_params, stream=None):
    p = np.ascontiguousarray(init_params, np.float32)
    assert p.size == kg_mlp_num_params(hidden)
    out = ctypes.c_void_p()
    _mcheck(_lib.kg_mlp_create(hidden, max_batch, p.ctypes.data, stream, ctypes.byref(out)), None)
    return out.value


def kg_mlp_destroy(m):
    _lib.kg_mlp_destroy(m)


def kg_mlp_set_norm(m, mean, stdev):
    a = np.ascontiguousarray(mean, np.float32)
    b = np.ascontiguousarray(stdev, np.float32)
    _mcheck(_lib.kg_mlp_set_norm(m, a.ctypes.data, b.ctypes.data), m)


def kg_mlp_get_params(m, hidden):
    out = np.empty(kg_mlp_num_params(hidden), np.float32)
    _mcheck(_lib.kg_mlp_get_params(m, out.ctypes.data), m)
    return out


def kg_mlp_forward(m, x_dev, out_dev):
    """x_dev: float32 cuda tensor [n, 4]; out_dev: float32 cuda tensor [n, 2]."""
    _mcheck(_lib.kg_mlp_forward(m, x_dev.data_ptr(), x_dev.shape[0], out_dev.data_ptr()), m)


def kg_mlp_grad(m, x_dev, y_dev, hidden):
    loss = np.empty(1, np.float32)
    g = np.empty(kg_mlp_num_params(hidden), np.float32)
    _mcheck(_lib.kg_mlp_grad(m, x_dev.data_ptr(), y_dev.data_ptr(), x_dev.shape[0],
                             loss.ctypes.data, g.ctypes.data), m)
    return float(loss[0]), g


def kg_mlp_train_step(m, x_dev, y_dev, lr, want_loss=False):
    loss = np.empty(1, np.float32)
    _mcheck(_lib.kg_mlp_train_step(m, x_dev.data_ptr(), y_dev.data_ptr(), x_dev.shape[0],
                                   ctypes.c_float(lr), loss.ctypes.data if want_loss else None), m)
    return float(loss[0]) if want_loss else None


def kg_mlp_forward_noalloc(hidden, params_dev, x_dev, out_dev, mean=None, stdev=None, stream=None):
    """Outputs for x_dev [n, 4] into out_dev [n, 2] (float32 cuda tensors)
    from parameters in the device tensor params_dev; allocates nothing."""
    m = None if mean is None else np.ascontiguousarray(mean, np.float32)
    s = None if stdev is None else np.ascontiguousarray(stdev, np.float32)
    st = _lib.kg_mlp_forward_noalloc(hidden, params_dev.data_ptr(),
                                     None if m is None else m.ctypes.data,
                                     None if s is None else s.ctypes.data,
                                     x_dev.data_ptr(), x_dev.shape[0], out_dev.data_ptr(), stream)
    if st != KG_OK:
        raise KGError(st, "kg_mlp_forward_noalloc")
