"""Python binding of libsedg (ctypes).  Argument marshalling only: every step of
the right-hand side and the Runge-Kutta stages runs in the library's HIP kernels.
Device memory comes from torch tensors (float64, contiguous, on the GPU) and
the stream from torch's current stream.

The functions mirror the C entry points declared in include/sedg.h:
sedg_create / sedg_destroy / sedg_init_state / sedg_rhs / sedg_max_dt / sedg_rk_step
/ sedg_diagnose / sedg_check / sedg_tables, the frozen map with its adjoint:
sedg_rhs_frozen / sedg_adjoint_rhs / sedg_tape_len / sedg_rk_step_tape /
sedg_rk_step_frozen / sedg_adjoint_rk_step, batched ensembles: sedg_batch_*, and
the right-hand side without device allocation: sedg_rhs_noalloc.  A missing or unloadable library raises at first use; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsedg.so")

SEDG_OK, SEDG_EINVAL, SEDG_EHIP, SEDG_ENOMEM, SEDG_ESTATE, SEDG_EUNSUPPORTED, SEDG_ESCRATCH = 0, -1, -2, -3, -4, -5, -6
SEDG_SSPRK3, SEDG_SSPRK54 = 0, 1

EXPORTED = ["sedg_create", "sedg_destroy", "sedg_state_len", "sedg_alpha_len", "sedg_set_params",
            "sedg_rhs", "sedg_max_dt", "sedg_rk_step", "sedg_check", "sedg_tables", "sedg_strerror",
            "sedg_profile", "sedg_profile_read", "sedg_rhs_frozen", "sedg_adjoint_rhs", "sedg_tape_len",
            "sedg_rk_step_tape", "sedg_adjoint_rk_step", "sedg_batch_create", "sedg_batch_destroy",
            "sedg_batch_state_len", "sedg_batch_state_offset", "sedg_batch_set_tuning", "sedg_batch_get_tuning",
            "sedg_batch_rk_step", "sedg_batch_check", "sedg_rhs_noalloc", "sedg_init_state", "sedg_diagnose",
            "sedg_rk_step_frozen", "sedg_refine", "sedg_coarsen", "sedg_nc_tables"]


class SedgError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code) if _lib else "error", code))


class Mesh_c(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("K", ctypes.c_int), ("nelem", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
                ("gamma", ctypes.c_double), ("family", ctypes.c_int)]


class Params_c(ctypes.Structure):
    _fields_ = [("tau_A", ctypes.c_double), ("tau_S", ctypes.c_double), ("alpha_H", ctypes.c_double),
                ("alpha_L", ctypes.c_double), ("beta_L", ctypes.c_double), ("cfl", ctypes.c_double),
                ("top_level", ctypes.c_int), ("level_mask", ctypes.c_uint), ("mode", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("sigma_floor", ctypes.c_double), ("integrator", ctypes.c_int)]


class Diag_c(ctypes.Structure):
    _fields_ = [("bulk_change", ctypes.c_double * 5), ("bulk_abs", ctypes.c_double * 5),
                ("alpha_bar_min", ctypes.c_double), ("alpha_bar_mean", ctypes.c_double),
                ("alpha_bar_max", ctypes.c_double), ("elems_by_lowest_order", ctypes.c_long * 4),
                ("squeezed", ctypes.c_long), ("beta_rejected", ctypes.c_long), ("fallbacks", ctypes.c_long)]


class Tuning_c(ctypes.Structure):
    _fields_ = [("epb4", ctypes.c_int), ("epb8", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("xcd_map", ctypes.c_int), ("waves_analyse", ctypes.c_int), ("waves_residual", ctypes.c_int)]


_lib = None


def load():
    """Load libsedg.so (raises OSError if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError("libsedg.so not built (run python -m paper_2011_03338_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.sedg_create.argtypes = [ctypes.POINTER(Mesh_c), ctypes.POINTER(Params_c), ctypes.POINTER(vp)]
    lib.sedg_destroy.argtypes = [vp]
    lib.sedg_state_len.argtypes = [vp]
    lib.sedg_state_len.restype = ctypes.c_long
    lib.sedg_alpha_len.argtypes = [vp]
    lib.sedg_alpha_len.restype = ctypes.c_long
    lib.sedg_set_params.argtypes = [vp, ctypes.POINTER(Params_c)]
    lib.sedg_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.sedg_max_dt.argtypes = [vp, vp, vp, vp]
    lib.sedg_rk_step.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp, vp, vp]
    lib.sedg_init_state.argtypes = [vp, vp, dp, ctypes.POINTER(ctypes.c_long)]
    lib.sedg_diagnose.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Diag_c), vp]
    lib.sedg_rk_step_frozen.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    lib.sedg_check.argtypes = [vp, ctypes.POINTER(ctypes.c_long)]
    lib.sedg_tables.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
    lib.sedg_profile.argtypes = [vp, ctypes.c_int]
    lib.sedg_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_long)]
    lib.sedg_rhs_frozen.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sedg_adjoint_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.sedg_tape_len.argtypes = [vp]
    lib.sedg_tape_len.restype = ctypes.c_long
    lib.sedg_rk_step_tape.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    lib.sedg_adjoint_rk_step.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    lib.sedg_batch_create.argtypes = [ctypes.POINTER(Mesh_c), ctypes.c_int, ctypes.POINTER(Params_c), ctypes.POINTER(vp)]
    lib.sedg_batch_destroy.argtypes = [vp]
    lib.sedg_batch_state_len.argtypes = [vp]
    lib.sedg_batch_state_len.restype = ctypes.c_long
    lib.sedg_batch_state_offset.argtypes = [vp, ctypes.c_int]
    lib.sedg_batch_state_offset.restype = ctypes.c_long
    lib.sedg_batch_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning_c)]
    lib.sedg_batch_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning_c)]
    lib.sedg_batch_rk_step.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp, vp]
    lib.sedg_batch_check.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_long)]
    lib.sedg_rhs_noalloc.argtypes = [ctypes.POINTER(Mesh_c), ctypes.POINTER(Params_c), vp, vp, vp, vp]
    lib.sedg_refine.argtypes = [vp, vp, vp, vp, vp]
    lib.sedg_coarsen.argtypes = [vp, vp, vp, vp, vp]
    lib.sedg_nc_tables.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
    lib.sedg_strerror.argtypes = [ctypes.c_int]
    lib.sedg_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().sedg_strerror(code).decode()


def _check(rc, what):
    if rc != SEDG_OK:
        raise SedgError(rc, what)


def mesh_c(m) -> Mesh_c:
    ne, lo, hi, bc = m.full()
    s = Mesh_c()
    s.dim, s.K = m.dim, m.K
    for a in range(3):
        s.nelem[a], s.lo[a], s.hi[a], s.bc[a] = ne[a], lo[a], hi[a], bc[a]
    s.gamma, s.family = m.gamma, m.family
    return s


def params_c(p) -> Params_c:
    s = Params_c()
    s.tau_A, s.tau_S, s.alpha_H, s.alpha_L, s.beta_L, s.cfl = p.tau_A, p.tau_S, p.alpha_H, p.alpha_L, p.beta_L, p.cfl
    s.top_level, s.level_mask, s.mode = p.top_level, p.level_mask, p.mode
    s.seed = int(getattr(p, "seed", 0))
    s.sigma_floor = float(getattr(p, "sigma_floor", 0.0))
    s.integrator = int(getattr(p, "integrator", 0))
    return s


def tables(n: int, family: int = 0) -> dict:
    """The library's own operator tables (host, no GPU needed)."""
    buf = np.zeros(16 * 64)
    cnt = load().sedg_tables(n, family, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size)
    if cnt < 0:
        raise SedgError(cnt, "sedg_tables")
    out, o = {}, 0
    for name, size, shp in [("xi", n, (n,)), ("w", n, (n,)), ("Dcal", n * n, (n, n)), ("D", n * n, (n, n)),
                            ("bm", n, (n,)), ("bp", n, (n,)), ("P", n * n, (n, n)), ("R", n * n, (n, n)),
                            ("Dhat", n * n, (n, n)), ("Bhl", n, (n,)), ("Bhr", n, (n,)),
                            ("Ip", n * n, (n, n)), ("Im", n * n, (n, n))]:
        out[name] = buf[o:o + size].reshape(shp).copy()
        o += size
    return out


def nc_tables(n: int, family: int = 0) -> dict:
    """The library's refinement / coarsening / mortar tables of level n (host)."""
    buf = np.zeros(8 * 64)
    cnt = load().sedg_nc_tables(n, family, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size)
    if cnt < 0:
        raise SedgError(cnt, "sedg_nc_tables")
    h = n // 2
    o = [0, 2 * n * n, 2 * n * n + h * n, 3 * n * n + h * n, 4 * n * n + h * n]
    return {"Z": buf[o[0]:o[1]].reshape(2 * n, n).copy(), "Q": buf[o[1]:o[2]].reshape(h, n).copy(),
            "Lm": buf[o[2]:o[3]].reshape(n, n).copy(), "Lp": buf[o[3]:o[4]].reshape(n, n).copy()}


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous(), "expected a contiguous float64 GPU tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def rhs_noalloc(mesh, params, u, dudt, bad=None, stream=None):
    """sedg_rhs_noalloc: the right-hand side without a context and without device
    allocation (work arrays in the library's static device array).  bad: optional
    int32 GPU tensor of one element receiving a bad element index (INT_MAX if none)."""
    if bad is not None:
        import torch
        assert bad.dtype == torch.int32 and bad.is_cuda and bad.numel() >= 1
    _check(load().sedg_rhs_noalloc(ctypes.byref(mesh_c(mesh)), ctypes.byref(params_c(params)), _ptr(u), _ptr(dudt),
                                   None if bad is None else ctypes.c_void_p(bad.data_ptr()), _stream(stream)),
           "sedg_rhs_noalloc")


class Solver:
    """One mesh/parameter context of the library on the current GPU."""

    def __init__(self, mesh, params):
        lib = load()
        self.mesh, self.params = mesh, params
        h = ctypes.c_void_p()
        _check(lib.sedg_create(ctypes.byref(mesh_c(mesh)), ctypes.byref(params_c(params)), ctypes.byref(h)),
               "sedg_create")
        self._h = h
        self.state_len = lib.sedg_state_len(h)
        self.alpha_len = lib.sedg_alpha_len(h)

    def close(self):
        if getattr(self, "_h", None):
            load().sedg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        self.params = params
        _check(load().sedg_set_params(self._h, ctypes.byref(params_c(params))), "sedg_set_params")

    def rhs(self, u, dudt, alpha_out=None, beta_out=None, alpha_in=None, stream=None):
        _check(load().sedg_rhs(self._h, _ptr(u), _ptr(dudt), _ptr(alpha_out), _ptr(beta_out), _ptr(alpha_in),
                               _stream(stream)), "sedg_rhs")

    def max_dt(self, u, dt_out, stream=None):
        _check(load().sedg_max_dt(self._h, _ptr(u), _ptr(dt_out), _stream(stream)), "sedg_max_dt")

    def rk_step(self, u, nsteps, dt_fixed=0.0, dt_log=None, alpha_log=None, stream=None):
        """nsteps steps of the context's integrator (SSP-RK3 or SSP-RK(5,4)) of u in place;
        dt_log (nsteps) and alpha_log (stages * nsteps * alpha_len, step-major) optionally
        receive the step sizes and every stage's factors."""
        _check(load().sedg_rk_step(self._h, _ptr(u), int(nsteps), float(dt_fixed), _ptr(dt_log), _ptr(alpha_log),
                                   _stream(stream)), "sedg_rk_step")

    def init_state(self, u_dev, u_host):
        """Copy a host state (numpy float64, state layout) into u_dev and check it; raises
        SedgError(SEDG_ESTATE) naming the first bad element."""
        import numpy as _np
        h = _np.ascontiguousarray(u_host, dtype=_np.float64)
        assert h.size == self.state_len and u_dev.numel() == self.state_len
        bad = ctypes.c_long(-1)
        rc = load().sedg_init_state(self._h, _ptr(u_dev), h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.byref(bad))
        if rc == SEDG_ESTATE:
            err = SedgError(rc, "sedg_init_state: element %d" % bad.value)
            err.element = bad.value
            raise err
        _check(rc, "sedg_init_state")

    def diagnose(self, u, dudt, alpha_bar=None, stream=None) -> dict:
        """Right-hand side at u into dudt plus its diagnostics (sedg_diagnose)."""
        d = Diag_c()
        _check(load().sedg_diagnose(self._h, _ptr(u), _ptr(dudt), _ptr(alpha_bar), ctypes.byref(d), _stream(stream)),
               "sedg_diagnose")
        nv = self.mesh.nvar
        return {"bulk_change": list(d.bulk_change)[:nv], "bulk_abs": list(d.bulk_abs)[:nv],
                "alpha_bar_min": d.alpha_bar_min, "alpha_bar_mean": d.alpha_bar_mean, "alpha_bar_max": d.alpha_bar_max,
                "elems_by_lowest_order": dict(zip(["FV", "O2", "O4", "O8"], list(d.elems_by_lowest_order))),
                "squeezed": d.squeezed, "beta_rejected": d.beta_rejected, "fallbacks": d.fallbacks}

    def rk_step_frozen(self, u, dt_dev, factors, stream=None):
        """len(dt_dev) steps of the frozen map, u in place; factors holds per step the
        [alpha x 3 | beta x 3] block of its tape (6 * alpha_len doubles per step)."""
        n = dt_dev.numel()
        assert factors.numel() >= n * 6 * self.alpha_len
        _check(load().sedg_rk_step_frozen(self._h, _ptr(u), n, _ptr(dt_dev), _ptr(factors), _stream(stream)),
               "sedg_rk_step_frozen")

    def rhs_frozen(self, u, alpha, beta, dudt, stream=None):
        """Right-hand side with alpha and beta held fixed."""
        _check(load().sedg_rhs_frozen(self._h, _ptr(u), _ptr(alpha), _ptr(beta), _ptr(dudt), _stream(stream)),
               "sedg_rhs_frozen")

    def adjoint_rhs(self, u, alpha, beta, lam, lam_out, stream=None):
        """lam_out = (dL/du)^T lam of the frozen right-hand side at u."""
        _check(load().sedg_adjoint_rhs(self._h, _ptr(u), _ptr(alpha), _ptr(beta), _ptr(lam), _ptr(lam_out),
                                       _stream(stream)), "sedg_adjoint_rhs")

    @property
    def tape_len(self) -> int:
        return load().sedg_tape_len(self._h)

    def rk_step_tape(self, u, dt_dev, tapes, stream=None):
        """len(dt_dev) SSP-RK3 steps of u in place, step j with step size dt_dev[j] (GPU
        tensor, e.g. a slice of a step-size log), recording tapes[j] (rows of tape_len)."""
        n = dt_dev.numel()
        assert tapes.numel() >= n * self.tape_len
        _check(load().sedg_rk_step_tape(self._h, _ptr(u), n, _ptr(dt_dev), _ptr(tapes), _stream(stream)),
               "sedg_rk_step_tape")

    def adjoint_rk_step(self, tapes, dt_dev, lam, stream=None):
        """lam <- (du_end/du_start)^T lam over the len(dt_dev) steps recorded in tapes."""
        n = dt_dev.numel()
        assert tapes.numel() >= n * self.tape_len
        _check(load().sedg_adjoint_rk_step(self._h, _ptr(tapes), n, _ptr(dt_dev), _ptr(lam), _stream(stream)),
               "sedg_adjoint_rk_step")

    def profile(self, on: bool):
        _check(load().sedg_profile(self._h, 1 if on else 0), "sedg_profile")

    def profile_read(self):
        """{kernel: (total_ms, launches)} for analyse, residual, step_size, faces."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_long * 4)()
        _check(load().sedg_profile_read(self._h, ms, cnt), "sedg_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(["analyse", "residual", "step_size", "faces"])}

    def refine(self, u, alpha, u_fine, stream=None):
        """Blended refinement of every element into 2^dim children (sedg_refine): u_fine is
        the state of the mesh with twice the elements per axis."""
        _check(load().sedg_refine(self._h, _ptr(u), _ptr(alpha), _ptr(u_fine), _stream(stream)), "sedg_refine")

    def coarsen(self, u_fine, alpha_fine, u, stream=None):
        """Blended coarsening of the doubled mesh's state onto this mesh (sedg_coarsen)."""
        _check(load().sedg_coarsen(self._h, _ptr(u_fine), _ptr(alpha_fine), _ptr(u), _stream(stream)),
               "sedg_coarsen")

    def check(self):
        """Returns -1, or raises SedgError(SEDG_ESTATE) naming the bad element."""
        bad = ctypes.c_long(0)
        rc = load().sedg_check(self._h, ctypes.byref(bad))
        if rc == SEDG_ESTATE:
            raise SedgError(rc, "sedg_check: element %d" % bad.value)
        _check(rc, "sedg_check")
        return -1


class BatchSolver:
    """An ensemble of independent 2-D problems advanced together (sedg_batch_*)."""

    def __init__(self, meshes, params):
        lib = load()
        self.meshes, self.params = list(meshes), params
        arr = (Mesh_c * len(self.meshes))(*[mesh_c(m) for m in self.meshes])
        h = ctypes.c_void_p()
        _check(lib.sedg_batch_create(arr, len(self.meshes), ctypes.byref(params_c(params)), ctypes.byref(h)),
               "sedg_batch_create")
        self._h = h
        self.state_len = lib.sedg_batch_state_len(h)
        self.offsets = [lib.sedg_batch_state_offset(h, p) for p in range(len(self.meshes))]

    @property
    def count(self) -> int:
        return len(self.meshes)

    def close(self):
        if getattr(self, "_h", None):
            load().sedg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, epb4=4, epb8=1, blocks_per_cu=0, xcd_map=1, waves_analyse=3, waves_residual=3):
        t = Tuning_c(epb4, epb8, blocks_per_cu, xcd_map, waves_analyse, waves_residual)
        _check(load().sedg_batch_set_tuning(self._h, ctypes.byref(t)), "sedg_batch_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning_c()
        _check(load().sedg_batch_get_tuning(self._h, ctypes.byref(t)), "sedg_batch_get_tuning")
        return {"epb4": t.epb4, "epb8": t.epb8, "blocks_per_cu": t.blocks_per_cu, "xcd_map": t.xcd_map,
                "waves_analyse": t.waves_analyse, "waves_residual": t.waves_residual}

    def pack(self, states):
        """One ensemble state (GPU tensor) from per-problem states (arrays or tensors),
        copied piece by piece."""
        import torch
        u = torch.empty(self.state_len, dtype=torch.float64, device="cuda")
        for x, m, o in zip(states, self.meshes, self.offsets):
            n = m.nvar * m.dof
            u[o:o + n].copy_(torch.as_tensor(x, dtype=torch.float64).reshape(-1))
        return u

    def views(self, u):
        """Per-problem views of an ensemble state, each shaped (nvar, gz, gy, gx)."""
        out = []
        for m, o in zip(self.meshes, self.offsets):
            n = m.nvar * m.dof
            out.append(u[o:o + n].view(*m.shape()))
        return out

    def rk_step(self, u, nsteps, dt_fixed=0.0, dt_log=None, stream=None):
        _check(load().sedg_batch_rk_step(self._h, _ptr(u), int(nsteps), float(dt_fixed), _ptr(dt_log),
                                         _stream(stream)), "sedg_batch_rk_step")

    def check(self):
        """Returns None, or raises SedgError(SEDG_ESTATE) naming the problem and element."""
        p = ctypes.c_int(-1)
        e = ctypes.c_long(-1)
        rc = load().sedg_batch_check(self._h, ctypes.byref(p), ctypes.byref(e))
        if rc == SEDG_ESTATE:
            err = SedgError(rc, "sedg_batch_check: problem %d element %d" % (p.value, e.value))
            err.problem, err.element = p.value, e.value
            raise err
        _check(rc, "sedg_batch_check")
        return None
