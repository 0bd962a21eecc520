"""Seeded synthetic inputs for the blended DG/FV solver.

This module holds problem descriptions (mesh, parameters) and initial states
only; it contains none of the scheme's arithmetic.  Both the HIP library and
the CPU oracle receive the arrays built here.

Initial states are subcell mean values of the conserved variables
(rho, rho*v, E) on the global subcell grid, laid out as u[var][z][y][x] with x
fastest.  Means are exact where the initial condition is separable (products
of 1-D integrals in closed form); otherwise they come from a tensor
Gauss-Legendre rule per subcell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

PERIODIC, OUTFLOW = 0, 1
GAUSS, LGL = 0, 1
ADAPTIVE, FORCE_DG, FORCE_FV, EXTERNAL, RANDOM = 0, 1, 2, 3, 4


@dataclasses.dataclass
class Mesh:
    dim: int
    K: int
    nelem: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc: Sequence[int]
    gamma: float = 1.4
    family: int = GAUSS

    def full(self):
        ne = list(self.nelem) + [1] * (3 - len(self.nelem))
        lo = list(self.lo) + [0.0] * (3 - len(self.lo))
        hi = list(self.hi) + [1.0] * (3 - len(self.hi))
        bc = list(self.bc) + [PERIODIC] * (3 - len(self.bc))
        return ne, lo, hi, bc

    @property
    def nvar(self) -> int:
        return self.dim + 2

    @property
    def grid(self):
        """Global subcell extents (gx, gy, gz)."""
        ne, _, _, _ = self.full()
        return [ne[a] * self.K if a < self.dim else 1 for a in range(3)]

    @property
    def dof(self) -> int:
        g = self.grid
        return g[0] * g[1] * g[2]

    @property
    def nel(self) -> int:
        ne, _, _, _ = self.full()
        return ne[0] * ne[1] * ne[2]

    def shape(self):
        g = self.grid
        return (self.nvar, g[2], g[1], g[0])

    def edges(self, a: int) -> np.ndarray:
        """Subcell edge coordinates along axis a."""
        ne, lo, hi, _ = self.full()
        n = ne[a] * self.K if a < self.dim else 1
        return np.linspace(lo[a], hi[a], n + 1)


@dataclasses.dataclass
class Params:
    tau_A: float = 100.0
    tau_S: float = 0.05
    alpha_H: float = 0.99
    alpha_L: float = 0.01
    beta_L: float = 0.95
    cfl: float = 0.5
    top_level: int = 0          # 0 -> K
    level_mask: int = 0         # 0 -> all levels
    mode: int = ADAPTIVE
    seed: int = 0               # RANDOM mode: generator seed
    sigma_floor: float = 0.0    # indicator denominator floor; 0 -> the paper's 1
    integrator: int = 0         # 0: SSP-RK3, 1: SSP-RK(5,4)


def alpha_len(mesh: Mesh, params: Params) -> int:
    top = params.top_level or mesh.K
    n, tot = top, 0
    while n >= 2:
        tot += (mesh.K // n) ** mesh.dim
        n //= 2
    return tot


# ---------------------------------------------------------------------------
# exact 1-D cell means of simple profiles
# ---------------------------------------------------------------------------

def _mean_sin(e: np.ndarray, k: float, phase: float = 0.0) -> np.ndarray:
    """Mean of sin(k x + phase) over the cells with edges e."""
    a, b = e[:-1], e[1:]
    return (np.cos(k * a + phase) - np.cos(k * b + phase)) / (k * (b - a))


def _mean_gauss(e: np.ndarray, c: float, s: float) -> np.ndarray:
    """Mean of exp(-(x-c)^2 / (2 s^2)) over the cells with edges e."""
    from scipy.special import erf
    a, b = e[:-1], e[1:]
    r = math.sqrt(2.0) * s
    return s * math.sqrt(math.pi / 2.0) * (erf((b - c) / r) - erf((a - c) / r)) / (b - a)


def _frac_right(e: np.ndarray, xj: float) -> np.ndarray:
    """Fraction of each cell lying at x >= xj."""
    a, b = e[:-1], e[1:]
    return np.clip((b - xj) / (b - a), 0.0, 1.0)


def _int_sin_right(e: np.ndarray, k: float, xj: float) -> np.ndarray:
    """(1/|cell|) * integral of sin(k x) over the part of each cell at x >= xj."""
    a, b = e[:-1], e[1:]
    lo = np.maximum(a, xj)
    val = np.where(b > lo, (np.cos(k * lo) - np.cos(k * b)) / k, 0.0)
    return val / (b - a)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def density_wave(mesh: Mesh, t: float = 0.0, vel=(0.1, 0.1, 0.1), amp=0.2, p0=1.0, gamma=1.4):
    """rho = 1 + amp * prod_a sin(2 pi (x_a - v_a t)), constant velocity and pressure:
    an exact solution of the Euler equations on the periodic unit box."""
    dim = mesh.dim
    k = 2.0 * math.pi
    m = [_mean_sin(mesh.edges(a), k, -k * vel[a] * t) for a in range(dim)]
    prod = m[0][None, None, :]
    if dim > 1:
        prod = prod * m[1][None, :, None]
    if dim > 2:
        prod = prod * m[2][:, None, None]
    g = mesh.grid
    rho = np.broadcast_to(1.0 + amp * prod, (g[2], g[1], g[0])).copy()
    u = np.zeros(mesh.shape())
    u[0] = rho
    v2 = 0.0
    for a in range(dim):
        u[1 + a] = vel[a] * rho
        v2 += vel[a] ** 2
    u[dim + 1] = p0 / (gamma - 1.0) + 0.5 * v2 * rho
    return u


def config0(seed: int = 0, nelem: int = 16, K: int = 4):
    """2-D periodic [0,1]^2, rho = 1 + 0.2 sin(2 pi x) sin(2 pi y), u = v = 0.1,
    p = 1, with rho and p doubled for x >= x_J (x_J ~ U(0.25, 0.75), seeded)."""
    rng = np.random.default_rng(seed)
    xj = float(rng.uniform(0.25, 0.75))
    mesh = Mesh(2, K, [nelem, nelem], [0.0, 0.0], [1.0, 1.0], [PERIODIC, PERIODIC])
    k = 2.0 * math.pi
    ex, ey = mesh.edges(0), mesh.edges(1)
    sx, sy = _mean_sin(ex, k), _mean_sin(ey, k)
    fr = _frac_right(ex, xj)
    sxr = _int_sin_right(ex, k, xj)
    # mean of rho * (1 + H(x - xj)) and of p * (1 + H(x - xj))
    rho = (1.0 + fr)[None, :] + 0.2 * (sx + sxr)[None, :] * sy[:, None]
    p = np.broadcast_to((1.0 + fr)[None, :], rho.shape)
    u = np.zeros(mesh.shape())
    u[0, 0] = rho
    u[1, 0] = 0.1 * rho
    u[2, 0] = 0.1 * rho
    u[3, 0] = p / 0.4 + 0.5 * 0.02 * rho
    return mesh, u, {"x_jump": xj}


def sedov(seed: int = 0, nelem: int = 256, K: int = 8, E: Optional[float] = None, rc: float = 0.1,
          p0: float = 1e-5, sigma: float = 0.06, L: float = 1.5):
    """2-D Sedov-type blast on [-L, L]^2 with outflow boundaries: rho = 1, v = 0,
    E = p0/(gamma-1) + E/(2 pi sigma^2) exp(-|x-c|^2/(2 sigma^2)), the centre c
    uniform in the disc |c| <= rc (seeded)."""
    rng = np.random.default_rng(seed)
    r = rc * math.sqrt(float(rng.uniform()))
    th = float(rng.uniform(0.0, 2.0 * math.pi))
    c = (r * math.cos(th), r * math.sin(th))
    Eb = 1.0 if E is None else E
    mesh = Mesh(2, K, [nelem, nelem], [-L, -L], [L, L], [OUTFLOW, OUTFLOW])
    gx = _mean_gauss(mesh.edges(0), c[0], sigma)
    gy = _mean_gauss(mesh.edges(1), c[1], sigma)
    u = np.zeros(mesh.shape())
    u[0, 0] = 1.0
    u[3, 0] = p0 / 0.4 + Eb / (2.0 * math.pi * sigma ** 2) * gy[:, None] * gx[None, :]
    return mesh, u, {"center": c, "E": Eb}


def pressure_pulse(seed: int = 0, nelem: int = 128, K: int = 8):
    """Config-0 state on [0,1]^2 plus a Gaussian pressure pulse of amplitude 5 and
    width 0.05 at a seeded centre c ~ U[0.25, 0.75]^2."""
    rng = np.random.default_rng(seed)
    mesh, u, info = config0(seed, nelem, K)
    c = rng.uniform(0.25, 0.75, size=2)
    gx = _mean_gauss(mesh.edges(0), float(c[0]), 0.05)
    gy = _mean_gauss(mesh.edges(1), float(c[1]), 0.05)
    u[3, 0] += 5.0 * gy[:, None] * gx[None, :] / 0.4
    info["pulse_center"] = tuple(float(x) for x in c)
    return mesh, u, info


def shear_layer_3d(seed: int = 0, nelem: int = 64, K: int = 8, nq: int = 3, device: str = "cpu"):
    """3-D Kelvin-Helmholtz layer on [-1,1]^3, periodic: rho = 0.5 + 0.25 [tanh((y+1/2)/0.05)
    - tanh((y-1/2)/0.05)], u = -0.5 + 0.5 [same], w = 0, p = 2.5 and
    v = (0.01/sqrt 8) sum_m sin(pi k_m.x + phi_m) with 8 seeded modes |k_m|_inf <= 4.
    Means by an nq^3 Gauss rule per subcell, computed with torch on `device`."""
    import torch
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < 8:
        k = rng.integers(-4, 5, size=3)
        if np.any(k != 0):
            ks.append(k)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=8)
    mesh = Mesh(3, K, [nelem] * 3, [-1.0] * 3, [1.0] * 3, [PERIODIC] * 3)
    G = mesh.grid[0]
    h = 2.0 / G
    xg, wg = np.polynomial.legendre.leggauss(nq)
    xg, wg = 0.5 * xg, 0.5 * wg
    dev = torch.device(device)
    dt = torch.float64
    cen = -1.0 + h * (torch.arange(G, dtype=dt, device=dev) + 0.5)
    out = torch.zeros((5, G, G, G), dtype=dt, device=dev)
    gam = 1.4
    for qz in range(nq):
        z = (cen + h * xg[qz]).view(G, 1, 1)
        for qy in range(nq):
            y = (cen + h * xg[qy]).view(1, G, 1)
            prof = torch.tanh((y + 0.5) / 0.05) - torch.tanh((y - 0.5) / 0.05)
            rho = 0.5 + 0.25 * prof
            uu = -0.5 + 0.5 * prof
            for qx in range(nq):
                x = (cen + h * xg[qx]).view(1, 1, G)
                w = float(wg[qx] * wg[qy] * wg[qz])
                v = torch.zeros((G, G, G), dtype=dt, device=dev)
                for m in range(8):
                    v += torch.sin(math.pi * (float(ks[m][0]) * x + float(ks[m][1]) * y + float(ks[m][2]) * z) + float(ph[m]))
                v *= 0.01 / math.sqrt(8.0)
                out[0] += w * rho.expand(G, G, G)
                out[1] += w * (rho * uu).expand(G, G, G)
                out[2] += w * (rho * v)
                out[4] += w * (2.5 / (gam - 1.0) + 0.5 * rho * (uu * uu + v * v))
    return mesh, out, {"modes": [k.tolist() for k in ks], "phases": ph.tolist()}


def ensemble(seed: int = 0, count: int = 256, sides=(32, 48, 64, 96, 128), Ks=(4, 8)):
    """Descriptions of independent Sedov-type blasts with seeded mesh side, K,
    blast energy in [0.5, 2] and centre within 0.2 of the origin."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(rng.choice(sides))
        K = int(rng.choice(Ks))
        E = float(rng.uniform(0.5, 2.0))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append({"side": side, "K": K, "E": E, "seed": sub_seed})
    return out


def ensemble_problem(desc):
    """The mesh and initial state of one ensemble member: the 2-D blast of sedov()
    on desc["side"]^2 elements with K = desc["K"], energy desc["E"] and a seeded
    centre within 0.2 of the origin."""
    return sedov(desc["seed"], desc["side"], desc["K"], E=desc["E"], rc=0.2)


def _tube_mesh(nelem: int, K: int, lo: float, hi: float, dim: int) -> Mesh:
    """1-D tube mesh (dim 1), or the same tube as a 2-D strip of nelem x 1 elements,
    outflow in x and periodic in y, every row of subcells evolving as the 1-D problem."""
    if dim == 1:
        return Mesh(1, K, [nelem], [lo], [hi], [OUTFLOW])
    return Mesh(2, K, [nelem, 1], [lo, 0.0], [hi, (hi - lo) / nelem], [OUTFLOW, PERIODIC])


def _tube_state(mesh: Mesh, rho, m, E) -> np.ndarray:
    u = np.zeros(mesh.shape())
    u[0, 0] = np.asarray(rho)[None, :]
    u[1, 0] = np.asarray(m)[None, :]
    u[mesh.dim + 1, 0] = np.asarray(E)[None, :]
    return u


def riemann_tube(left, right, x_d: float, T: float, nelem: int = 32, K: int = 8, lo: float = 0.0,
                 hi: float = 1.0, dim: int = 2, gamma: float = 1.4):
    """Riemann problem (rho, v, p) = left for x < x_d, right for x >= x_d; cell means exact
    (the diaphragm may cut a subcell)."""
    mesh = _tube_mesh(nelem, K, lo, hi, dim)
    fr = _frac_right(mesh.edges(0), x_d)

    def cons(st):
        rho, v, p = st
        return rho, rho * v, p / (gamma - 1.0) + 0.5 * rho * v * v

    cl, cr = cons(left), cons(right)
    u = _tube_state(mesh, *[(1.0 - fr) * a + fr * b for a, b in zip(cl, cr)])
    return mesh, u, {"x_diaphragm": x_d, "T": T, "left": tuple(left), "right": tuple(right)}


def sod_tube(nelem: int = 32, K: int = 8, dim: int = 2):
    """Sod shock tube on [0, 1] (Sec. 3.4): diaphragm at x = 0.5; (rho, v, p) = (1, 0, 1)
    left, (0.125, 0, 0.1) right; final time 0.2.  The diaphragm falls on a subcell edge."""
    return riemann_tube((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.5, 0.2, nelem, K, dim=dim)


def lax_tube(nelem: int = 32, K: int = 8, dim: int = 2):
    """Lax shock tube on [0, 1] (Sec. 3.4): diaphragm at 0.5, (rho, v, p) =
    (0.445, 0.689, 3.528) left, (0.5, 0, 0.571) right, final time 0.15 (the values and
    the time the text prints)."""
    return riemann_tube((0.445, 0.689, 3.528), (0.5, 0.0, 0.571), 0.5, 0.15, nelem, K, dim=dim)


def shu_osher(nelem: int = 32, K: int = 8, dim: int = 2, gamma: float = 1.4):
    """Shu-Osher tube on [-4.5, 4.5] (Sec. 3.4): (rho, v, p) = (3.8567143, 2.629369,
    10.33333) for x < -4, (1 + 0.2 sin(5 x), 0, 1) beyond; final time 1.8.  Means exact:
    the subcell holding x = -4 is split, the sine integrated."""
    mesh = _tube_mesh(nelem, K, -4.5, 4.5, dim)
    e = mesh.edges(0)
    fr = _frac_right(e, -4.0)
    rl, vl, pl = 3.8567143, 2.629369, 10.33333
    rho = (1.0 - fr) * rl + fr * 1.0 + 0.2 * _int_sin_right(e, 5.0, -4.0)
    m = (1.0 - fr) * rl * vl
    E = (1.0 - fr) * (pl / (gamma - 1.0) + 0.5 * rl * vl * vl) + fr * (1.0 / (gamma - 1.0))
    return mesh, _tube_state(mesh, rho, m, E), {"T": 1.8}
