"""ctypes front end of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sedg_oracle.c")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("K", ctypes.c_int), ("nelem", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
                ("gamma", ctypes.c_double), ("family", ctypes.c_int)]


class _Params(ctypes.Structure):
    _fields_ = [("tau_A", ctypes.c_double), ("tau_S", ctypes.c_double), ("alpha_H", ctypes.c_double),
                ("alpha_L", ctypes.c_double), ("beta_L", ctypes.c_double), ("cfl", ctypes.c_double),
                ("top_level", ctypes.c_int), ("level_mask", ctypes.c_uint), ("mode", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("draw", ctypes.c_longlong), ("sigma_floor", ctypes.c_double),
                ("integrator", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.or_rhs.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, dp,
                                ctypes.POINTER(ctypes.c_long)]
        _lib.or_rhs.restype = ctypes.c_int
        _lib.or_max_dt.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp]
        _lib.or_max_dt.restype = ctypes.c_double
        _lib.or_rk3.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, ctypes.c_int, ctypes.c_double, dp]
        _lib.or_rk3.restype = ctypes.c_int
        _lib.or_tables.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
        _lib.or_tables.restype = ctypes.c_int
        _lib.or_alpha_len.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params)]
        _lib.or_num_threads.restype = ctypes.c_int
        _lib.or_alpha_bar.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, dp]
        _lib.or_alpha_bar.restype = ctypes.c_int
    return _lib


def _mesh(m) -> _Mesh:
    ne, lo, hi, bc = m.full()
    s = _Mesh()
    s.dim, s.K = m.dim, m.K
    for a in range(3):
        s.nelem[a], s.lo[a], s.hi[a], s.bc[a] = ne[a], lo[a], hi[a], bc[a]
    s.gamma, s.family = m.gamma, m.family
    return s


def _params(p, draw: int = 0) -> _Params:
    s = _Params()
    s.tau_A, s.tau_S, s.alpha_H, s.alpha_L, s.beta_L, s.cfl = p.tau_A, p.tau_S, p.alpha_H, p.alpha_L, p.beta_L, p.cfl
    s.top_level, s.level_mask, s.mode = p.top_level, p.level_mask, p.mode
    s.seed = int(getattr(p, "seed", 0))
    s.draw = int(draw)
    s.sigma_floor = float(getattr(p, "sigma_floor", 0.0))
    s.integrator = int(getattr(p, "integrator", 0))
    return s


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    pass


def tables(n: int, family: int = 0) -> dict:
    buf = np.zeros(16 * 64, dtype=np.float64)
    cnt = lib().or_tables(n, family, _ptr(buf), buf.size)
    if cnt < 0:
        raise OracleError("bad level")
    out, o = {}, 0
    for name, size, shp in [("xi", n, (n,)), ("w", n, (n,)), ("Dcal", n * n, (n, n)), ("D", n * n, (n, n)),
                            ("bm", n, (n,)), ("bp", n, (n,)), ("P", n * n, (n, n)), ("R", n * n, (n, n)),
                            ("Dhat", n * n, (n, n)), ("Bhl", n, (n,)), ("Bhr", n, (n,)),
                            ("Ip", n * n, (n, n)), ("Im", n * n, (n, n))]:
        out[name] = buf[o:o + size].reshape(shp).copy()
        o += size
    return out


def alpha_len(mesh, params) -> int:
    return lib().or_alpha_len(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)))


def rhs(mesh, params, u, alpha_in=None, full: bool = False, draw: int = 0):
    """One right-hand side.  Returns dudt, or (dudt, info) with full=True where info
    holds alpha, beta, xraw, araw (each nel x A) and the fallback count.  draw: index
    of the factor draw in RANDOM mode."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    A = alpha_len(mesh, params)
    nel = mesh.nel
    dudt = np.zeros_like(u)
    al = np.zeros((nel, A))
    be = np.zeros((nel, A))
    xr = np.zeros((nel, A))
    ar = np.zeros((nel, A))
    ain = None if alpha_in is None else np.ascontiguousarray(alpha_in, dtype=np.float64).reshape(nel, A)
    nfb = ctypes.c_long(0)
    rc = lib().or_rhs(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params, draw)), _ptr(u), _ptr(dudt),
                      _ptr(al), _ptr(be), _ptr(ain), _ptr(xr), _ptr(ar), ctypes.byref(nfb))
    if rc != 0:
        raise OracleError("or_rhs failed: %d" % rc)
    if full:
        return dudt, {"alpha": al, "beta": be, "xraw": xr, "araw": ar, "fallbacks": nfb.value}
    return dudt


def max_dt(mesh, params, u) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    dt = lib().or_max_dt(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(u))
    if dt <= 0:
        raise OracleError("bad state")
    return dt


def rk3(mesh, params, u, nsteps: int, dt_fixed: float = 0.0, draw: int = 0):
    """nsteps steps of SSP-RK3 (or SSP-RK(5,4) with params.integrator = 1); returns
    (u_new, dt_log).  In RANDOM mode the right-hand sides use draws draw, draw + 1, ...
    (one per stage)."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    dts = np.zeros(max(nsteps, 1))
    rc = lib().or_rk3(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params, draw)), _ptr(u), nsteps, dt_fixed,
                      _ptr(dts))
    if rc != 0:
        raise OracleError("or_rk3 failed: %d" % rc)
    return u, dts[:nsteps]


def alpha_bar(mesh, params, alpha):
    """Weighted blending factor of every subcell (eq. order-estimate), shaped (gz, gy, gx)."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    out = np.zeros(mesh.dof)
    rc = lib().or_alpha_bar(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(al), _ptr(out))
    if rc != 0:
        raise OracleError("or_alpha_bar failed: %d" % rc)
    g = mesh.grid
    return out.reshape(g[2], g[1], g[0])


def nc_tables(n: int, family: int = 0) -> dict:
    """Z = P^(n->2n), Q = P^(n->n/2) and the mortar matrices L_-, L_+ of level n."""
    L = lib()
    L.or_nc_tables.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    buf = np.zeros(8 * 64)
    if L.or_nc_tables(n, family, _ptr(buf), buf.size) < 0:
        raise OracleError("bad level")
    h = n // 2
    o = [0, 2 * n * n, 2 * n * n + h * n, 3 * n * n + h * n, 4 * n * n + h * n]
    return {"Z": buf[o[0]:o[1]].reshape(2 * n, n).copy(), "Q": buf[o[1]:o[2]].reshape(h, n).copy(),
            "Lm": buf[o[2]:o[3]].reshape(n, n).copy(), "Lp": buf[o[3]:o[4]].reshape(n, n).copy()}


def _setup_rc():
    L = lib()
    dp = ctypes.POINTER(ctypes.c_double)
    for f in (L.or_refine, L.or_coarsen):
        f.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, dp, dp]
        f.restype = ctypes.c_int
    return L


def fine_mesh(mesh):
    """The mesh with twice the elements per axis (same box, K and boundaries)."""
    import dataclasses
    ne = list(mesh.nelem)
    return dataclasses.replace(mesh, nelem=[2 * x for x in ne])


def refine(mesh, params, u, alpha):
    """Blended refinement (eq. 3D-refinement) of every element into 2^dim children:
    the state on fine_mesh(mesh)."""
    L = _setup_rc()
    u = np.ascontiguousarray(u, dtype=np.float64)
    fm = fine_mesh(mesh)
    out = np.zeros(fm.shape())
    rc = L.or_refine(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(u),
                     _ptr(np.ascontiguousarray(alpha, dtype=np.float64)), _ptr(out))
    if rc != 0:
        raise OracleError("or_refine failed: %d" % rc)
    return out


def coarsen(mesh, params, u_fine, alpha_fine):
    """Blended coarsening (eq. 3D-coarsening) of the state on fine_mesh(mesh) onto mesh."""
    L = _setup_rc()
    uf = np.ascontiguousarray(u_fine, dtype=np.float64)
    out = np.zeros(mesh.shape())
    rc = L.or_coarsen(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(uf),
                      _ptr(np.ascontiguousarray(alpha_fine, dtype=np.float64)), _ptr(out))
    if rc != 0:
        raise OracleError("or_coarsen failed: %d" % rc)
    return out


def num_threads() -> int:
    return lib().or_num_threads()


def _setup_frozen():
    L = lib()
    dp = ctypes.POINTER(ctypes.c_double)
    L.or_rhs_frozen.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, dp, dp, dp]
    L.or_rhs_frozen.restype = ctypes.c_int
    L.or_adjoint_rhs.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), dp, dp, dp, dp, dp]
    L.or_adjoint_rhs.restype = ctypes.c_int
    return L


def rhs_frozen(mesh, params, u, alpha, beta):
    """Right-hand side with the blending factors and squeezing parameters held fixed."""
    L = _setup_frozen()
    u = np.ascontiguousarray(u, dtype=np.float64)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros_like(u)
    rc = L.or_rhs_frozen(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(u), _ptr(al), _ptr(be), _ptr(out))
    if rc != 0:
        raise OracleError("or_rhs_frozen failed: %d" % rc)
    return out


def adjoint_rhs(mesh, params, u, alpha, beta, lam):
    """(dL/du)^T lam of the frozen right-hand side at u."""
    L = _setup_frozen()
    u = np.ascontiguousarray(u, dtype=np.float64)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros_like(u)
    rc = L.or_adjoint_rhs(ctypes.byref(_mesh(mesh)), ctypes.byref(_params(params)), _ptr(u), _ptr(al), _ptr(be),
                          _ptr(lam), _ptr(out))
    if rc != 0:
        raise OracleError("or_adjoint_rhs failed: %d" % rc)
    return out
