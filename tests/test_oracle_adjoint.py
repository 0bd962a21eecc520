"""Pins of the oracle's adjoint (vector-Jacobian product) of the frozen right-hand
side: the blending factors and squeezing parameters are held at their values at
the base state.  The adjoint takes its local Jacobians by forward-mode dual
numbers; it is checked against central differences of the oracle's forward map.

HLL-Einfeldt wave speeds are min/max of two estimates that coincide when the left
and right interface states are equal, so the frozen map has kinks wherever the
interface states of smooth data nearly agree; central differences straddle such
kinks; the interface-safety margins add further non-smooth points.  The
directional checks use states whose interface states differ (jumps, random
blends, FV-only) and a step of 1e-7 (relative), below the distance to those
points; the one kink case is checked with one-sided differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03338_amd import workloads as W


def _dot_check(mesh, u, alpha, beta, seed=0, eps=1e-7):
    p = W.Params()
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(u.shape) * np.abs(u)
    w = rng.standard_normal(u.shape)
    fd = (O.rhs_frozen(mesh, p, u + eps * v, alpha, beta) - O.rhs_frozen(mesh, p, u - eps * v, alpha, beta)) / (2 * eps)
    lhs = (w * fd).sum()
    rhs = (O.adjoint_rhs(mesh, p, u, alpha, beta, w) * v).sum()
    return abs(lhs - rhs) / abs(lhs)


def _base(mesh, u):
    d, info = O.rhs(mesh, W.Params(), u, full=True)
    return d, info["alpha"], info["beta"]


@pytest.mark.parametrize("K", [4, 8])
def test_frozen_map_equals_adaptive_at_base(K):
    mesh, u, _ = W.config0(2, 3, K)
    d, al, be = _base(mesh, u)
    assert np.array_equal(O.rhs_frozen(mesh, W.Params(), u, al, be), d)


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("mode", ["random", "fv"])
def test_adjoint_directional_2d(K, mode):
    mesh, u, _ = W.config0(1, 3, K)
    _, al, be = _base(mesh, u)
    if mode == "random":
        al = np.random.default_rng(5).uniform(0, 1, al.shape)
    else:
        al = np.zeros_like(al)
    assert _dot_check(mesh, u, al, be) < 1e-6


def test_adjoint_directional_adaptive_k4():
    mesh, u, _ = W.config0(1, 3, 4)
    _, al, be = _base(mesh, u)
    assert _dot_check(mesh, u, al, be) < 1e-6


def test_adjoint_directional_blast_with_squeezes():
    """Resolved blast: squeezed reconstructions (beta < 1), outflow boundaries."""
    mesh, u, _ = W.sedov(2, 6, 8, L=0.3, sigma=0.03)
    _, al, be = _base(mesh, u)
    assert np.any(be < 1.0)
    rng = np.random.default_rng(7)
    al = rng.uniform(0.2, 0.8, al.shape)
    assert _dot_check(mesh, u, al, be) < 1e-6
    assert _dot_check(mesh, u, np.zeros_like(al), be) < 1e-6


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("mode", ["random", "dg"])
def test_adjoint_directional_lgl(K, mode):
    """LGL sub-cells.  The config-0 state gets seeded 1e-3 relative noise: LGL nodes on
    the element faces sample its jump where the modulation vanishes, a pure contact
    whose two Einfeldt speed estimates coincide (a kink of the frozen map)."""
    import dataclasses
    mesh, u, _ = W.config0(1, 3, K)
    mesh = dataclasses.replace(mesh, family=W.LGL)
    u = u * (1.0 + 1e-3 * np.random.default_rng(7).standard_normal(u.shape))
    _, al, be = _base(mesh, u)
    al = np.random.default_rng(2).uniform(0, 1, al.shape) if mode == "random" else np.ones_like(al)
    assert _dot_check(mesh, u, al, be) < 1e-6


@pytest.mark.parametrize("dim,K", [(1, 8), (3, 4)])
def test_adjoint_directional_other_dims(dim, K):
    ne = {1: [5], 3: [2, 2, 2]}[dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [1] + [0] * (dim - 1))
    rng = np.random.default_rng(3)
    u = np.zeros(mesh.shape())
    u[0] = 1.0 + 0.5 * rng.uniform(size=u[0].shape)
    u[1] = 0.3 * u[0]
    u[dim + 1] = (1.0 + 0.5 * rng.uniform(size=u[0].shape)) / 0.4 + 0.5 * 0.09 * u[0]
    _, al, be = _base(mesh, u)
    al = rng.uniform(0, 1, al.shape)
    assert _dot_check(mesh, u, al, be) < 1e-6


def test_adjoint_rows_single_element_pure_dg():
    """One periodic K = 8 element, pure top-level DG: rows of the transposed Jacobian
    equal rows of a finite-difference Jacobian."""
    K = 8
    m = W.Mesh(2, K, [1, 1], [0, 0], [1, 1], [0, 0])
    u = W.density_wave(m, vel=(0.3, -0.2, 0), amp=0.2)
    p = W.Params()
    A = W.alpha_len(m, p)
    al = np.zeros((1, A))
    al[:, 0] = 1
    be = np.ones((1, A))
    uf = u.reshape(-1)
    n = uf.size
    for i in (0, 77, 200):
        lam = np.zeros(n)
        lam[i] = 1
        g = O.adjoint_rhs(m, p, u, al, be, lam.reshape(u.shape)).reshape(-1)
        row = np.zeros(n)
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1e-6 * max(abs(uf[j]), 1e-3)
            row[j] = (O.rhs_frozen(m, p, (uf + e).reshape(u.shape), al, be).reshape(-1)[i]
                      - O.rhs_frozen(m, p, (uf - e).reshape(u.shape), al, be).reshape(-1)[i]) / (2 * e[j])
        assert np.abs(g - row).max() <= 1e-6 * np.abs(row).max()


def test_adjoint_at_wave_speed_kink():
    """A diagonal entry next to nearly equal interface states (smooth neighbours):
    the two one-sided slopes differ at step 1e-4, agree at 1e-10, and the adjoint
    equals the one-sided slope at u."""
    m, u, _ = W.config0(1, 3, 8)
    p = W.Params()
    _, info_al, be = _base(m, u)
    al = np.zeros_like(info_al)
    al[:, 0] = 1
    uf = u.reshape(-1)
    G = m.grid
    i = 3 * G[0] + 3
    lam = np.zeros(uf.size)
    lam[i] = 1
    g = O.adjoint_rhs(m, p, u, al, be, lam.reshape(u.shape)).reshape(-1)[i]
    f0 = O.rhs_frozen(m, p, u, al, be).reshape(-1)[i]

    def one_sided(eps):
        e = np.zeros(uf.size)
        e[i] = eps * abs(uf[i])
        fp = O.rhs_frozen(m, p, (uf + e).reshape(u.shape), al, be).reshape(-1)[i]
        fm = O.rhs_frozen(m, p, (uf - e).reshape(u.shape), al, be).reshape(-1)[i]
        return (fp - f0) / e[i], (f0 - fm) / e[i]

    jp, jm = one_sided(1e-4)
    assert abs(jp - jm) > 1e-2 * abs(jp)          # a genuine kink nearby
    jp, jm = one_sided(1e-10)
    assert abs(jp - jm) <= 1e-5 * abs(jp)
    assert abs(g - 0.5 * (jp + jm)) <= 1e-5 * abs(g)
