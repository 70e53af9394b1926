"""A plan with its workspace held in a torch device tensor."""
import numpy as np
import torch

from . import kg as _kg


class Solver:
    """One Klein-Gordon run on the current GPU: owns a plan and its workspace.

    Work goes to torch's current stream at construction time.  Initial data
    may be numpy arrays (host) or contiguous float64 torch tensors on the GPU
    (complex128 for a complex field).
    """

    def __init__(self, n, dt, L=0.0, linear_only=False, blowup_threshold=0.0,
                 precision=_kg.KG_FP64, complex_field=False, dealias=False):
        """precision: KG_FP64 (0) or KG_FP32 (1).  complex_field: u is complex
        and the cubic term is |u|^2 u.  dealias: 2/3-rule truncation of the
        nonlinear term."""
        self.n = n
        self.complex_field = bool(complex_field)
        self.params = _kg.make_params(n, dt, L, precision, linear_only, blowup_threshold,
                                      complex_field, dealias)
        nbytes = _kg.kg_workspace_bytes(self.params)
        if nbytes == 0:
            raise _kg.KGError(_kg.KG_E_INVALID, f"unsupported parameters n={n}, dt={dt}")
        self.stream = torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.plan = _kg.kg_plan(self.params, self.workspace.data_ptr(), nbytes,
                                self.stream.cuda_stream)

    def close(self):
        if self.plan:
            self.stream.synchronize()
            _kg.kg_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_state(self, u0, aux=None, mode=_kg.KG_INIT_VELOCITY):
        for x in (u0, aux):
            if x is None:
                continue
            if isinstance(x, np.ndarray):
                ok = x.dtype == (np.complex128 if self.complex_field else np.float64)
            else:
                ok = x.dtype == (torch.complex128 if self.complex_field else torch.float64)
            if not ok:
                raise TypeError(f"initial data of dtype {x.dtype}; this run takes "
                                f"{'complex128' if self.complex_field else 'float64'}")
        _kg.kg_set_state(self.plan, u0, aux, mode)

    def step(self, nsteps, sync=True):
        return _kg.kg_step(self.plan, nsteps, _kg.KG_STEP_SYNC if sync else 0)

    def energy(self):
        return _kg.kg_energy(self.plan)

    def records(self, first, count):
        return _kg.kg_records(self.plan, first, count)

    def energies(self, first, count):
        return _kg.kg_energies(self.plan, first, count)

    def stats(self, max_abs_u=False):
        return _kg.kg_stats(self.plan, max_abs_u)

    def energy_alarm(self, rel_tol):
        """Stop the run once the energy drifts by more than rel_tol (0: off)."""
        _kg.kg_set_energy_alarm(self.plan, rel_tol)

    def state(self):
        """(u^{n-1}, u^n) on the host."""
        return _kg.kg_get_state(self.plan, self.n, complex_field=self.complex_field)

    def u(self, out=None):
        return _kg.kg_get_u(self.plan, self.n, out, self.complex_field)

    def spectrum(self, which=0):
        return _kg.kg_get_spectrum(self.plan, self.n, which, complex_field=self.complex_field)

    def save(self):
        return _kg.kg_save_state(self.plan)

    def load(self, buf):
        _kg.kg_load_state(self.plan, buf)
