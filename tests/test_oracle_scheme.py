"""Pins of the oracle's blended right-hand side against what the paper fixes:
the pure FV and pure DG limits (Sec. 2.5 remark), sub-element DGSEM, the 1-D
multi-level scheme (Sec. 2.6) written independently in matrix form,
conservation for arbitrary blending factors (Sec. 2.5 lemma, Sec. 3.3),
free-stream preservation, reductions in dimension, symmetry, the indicator's
closed cases (Sec. 2.7), the squeeze (Sec. 2.4) and convergence order."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03338_amd import workloads as W
from tests import refs

RNG = np.random.default_rng(1234)
# comparisons against references built from double-precision tables: rounding of the
# K = 8 operators (condition numbers ~10-30) reaches ~1e-12 of the largest output
TOL = 2e-11


def smooth_state(mesh, amp=0.2, seed=0):
    """Smooth, strictly permissible periodic state with nonzero velocity."""
    rng = np.random.default_rng(seed)
    u = W.density_wave(mesh, vel=(0.3, -0.2, 0.1), amp=amp)
    # add a smooth pressure/velocity variation through the energy and momenta
    g = mesh.grid
    xs = [0.5 * (mesh.edges(a)[1:] + mesh.edges(a)[:-1]) for a in range(3)]
    X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 3)
    bump = np.cos(2 * np.pi * X[2] + ph[0])
    if mesh.dim > 1:
        bump = bump * np.cos(2 * np.pi * X[1] + ph[1])
    u[mesh.dim + 1] += 0.1 * bump
    u[1] += 0.02 * bump * u[0]
    return u


def mesh2d(K, ne=(3, 2), bc=(0, 0), fam=0):
    return W.Mesh(2, K, list(ne), [0.0, 0.0], [1.0, 1.0], list(bc), family=fam)


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("bc", [0, 1])
def test_force_fv_is_first_order_fv(K, bc):
    """alpha = 0 everywhere recovers the subcell FV scheme (Sec. 2.5 remark)."""
    mesh = mesh2d(K, bc=(bc, bc))
    _, u, _ = W.config0(3, 2, K)
    mesh = W.Mesh(2, K, [2, 2], [0, 0], [1, 1], [bc, bc])
    p = W.Params(mode=W.FORCE_FV)
    d = O.rhs(mesh, p, u)
    r = refs.fv_rhs(mesh, u)
    assert np.abs(d - r).max() <= TOL * np.abs(r).max()


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("fam", [0, 1])
def test_force_dg_is_dgsem(K, bc, fam):
    """alpha = 1 at the top level recovers nodal DGSEM mapped to mean values (Sec. 2.5)."""
    mesh = mesh2d(K, bc=(bc, bc), fam=fam)
    u = smooth_state(mesh)
    p = W.Params(mode=W.FORCE_DG)
    d, info = O.rhs(mesh, p, u, full=True)
    assert np.all(info["beta"][:, 0] == 1.0)
    r = refs.dgsem_rhs(mesh, u, K, refs.np_tables(K, lobatto=bool(fam)))
    assert np.abs(d - r).max() <= TOL * np.abs(r).max()


@pytest.mark.parametrize("K,n", [(4, 2), (8, 4), (8, 2)])
def test_subelement_dgsem(K, n):
    """theta^(n) = 1 on every sub-element is DGSEM on the sub-element grid."""
    mesh = mesh2d(K)
    u = smooth_state(mesh)
    p = W.Params(mode=W.EXTERNAL)
    A = W.alpha_len(mesh, p)
    al = np.zeros((mesh.nel, A))
    # level order in the alpha vector: K, K/2, ..., 2
    off, m = 0, K
    while m >= 2:
        cnt = (K // m) ** 2
        if m == n:
            al[:, off:off + cnt] = 1.0
        off += cnt
        m //= 2
    d = O.rhs(mesh, p, u, alpha_in=al)
    r = refs.dgsem_rhs(mesh, u, n)
    assert np.abs(d - r).max() <= TOL * np.abs(r).max()


def _alpha_levels_1d(K, top=None):
    top = top or K
    lv, n = [], top
    while n >= 2:
        lv.append(n)
        n //= 2
    return lv


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("periodic", [True, False])
def test_multilevel_1d_matches_matrix_form(K, periodic):
    """Random blending factors on every level: the 1-D oracle equals the paper's
    matrix-form multi-level scheme (Sec. 2.6) built with independent tables."""
    ne = 5
    mesh = W.Mesh(1, K, [ne], [0.0], [1.0], [0 if periodic else 1])
    x = 0.5 * (mesh.edges(0)[1:] + mesh.edges(0)[:-1])
    rho = 1.0 + 0.3 * np.exp(-((x - 0.4) / 0.15) ** 2)
    v = 0.2 + 0.1 * np.sin(2 * np.pi * x)
    pr = 1.0 + 0.2 * np.cos(2 * np.pi * x)
    u = np.zeros(mesh.shape())
    u[0, 0, 0], u[1, 0, 0], u[2, 0, 0] = rho, rho * v, pr / 0.4 + 0.5 * rho * v * v
    levels = _alpha_levels_1d(K)
    p = W.Params(mode=W.EXTERNAL)
    A = W.alpha_len(mesh, p)
    al = RNG.uniform(0.05, 0.95, size=(ne, A))
    d, info = O.rhs(mesh, p, u, alpha_in=al, full=True)
    assert np.all(info["beta"] == 1.0) and info["fallbacks"] == 0
    alphas, off = {}, 0
    for n in levels:
        alphas[n] = al[:, off:off + K // n]
        off += K // n
    r = refs.ml1d_rhs(K, ne, 1.0 / ne, u[:, 0, 0, :], alphas, levels, periodic)
    assert np.abs(d[:, 0, 0, :] - r).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("K", [4, 8])
def test_multilevel_2d_brute_force_2x2(K):
    """Random blending factors on every level of a periodic 2x2-element mesh: the 2-D
    oracle equals a dense brute force of the multi-level scheme (Kronecker-assembled
    block-diagonal operators on the global grid, independent tables; Sec. 2.6 with the
    element-face fluxes of App. eqs. 3D-interface-fluxes / 3D-blend-interface-fluxes in
    d = 2).  Every face is partially blended.  Measured: 1.3e-14 (K = 4), 2.9e-13
    (K = 8, where the n = 8 reconstruction amplifies rounding)."""
    rng = np.random.default_rng(7 + K)
    ne = 2
    mesh = W.Mesh(2, K, [ne, ne], [0.0, 0.0], [1.0, 1.0], [0, 0])
    G = ne * K
    nz = 0.01 if K == 4 else 1e-4     # cell noise the degree K-1 reconstruction keeps positive
    xc = (np.arange(G) + 0.5) / G
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + nz * rng.uniform(-1, 1, (G, G))
    vx = 0.3 + 0.1 * np.cos(2 * np.pi * Y) + nz * rng.uniform(-1, 1, (G, G))
    vy = -0.2 + 0.1 * np.sin(2 * np.pi * X) + nz * rng.uniform(-1, 1, (G, G))
    pr = 1.0 + 0.2 * np.cos(2 * np.pi * (X + Y)) + nz * rng.uniform(-1, 1, (G, G))
    u = np.zeros(mesh.shape())
    u[0, 0], u[1, 0], u[2, 0] = rho, rho * vx, rho * vy
    u[3, 0] = pr / 0.4 + 0.5 * rho * (vx ** 2 + vy ** 2)
    p = W.Params(mode=W.EXTERNAL)
    al = rng.uniform(0.05, 0.95, size=(mesh.nel, W.alpha_len(mesh, p)))
    d, info = O.rhs(mesh, p, u, alpha_in=al, full=True)
    assert np.all(info["beta"] == 1.0) and info["fallbacks"] == 0
    r = refs.ml2d_rhs(K, ne, 1.0 / ne, u[:, 0], al, _alpha_levels_1d(K))
    for v in range(4):
        assert np.abs(d[v, 0] - r[v]).max() <= 1e-12 * np.abs(r[v]).max(), v


@pytest.mark.parametrize("dim,K", [(1, 8), (2, 4), (2, 8), (3, 4)])
def test_conservation_random_alpha(dim, K):
    """Any blending factors: the domain integral of the right-hand side vanishes on a
    periodic mesh (lemma of Sec. 2.5, conservation test of Sec. 3.3)."""
    ne = {1: [6], 2: [3, 2], 3: [2, 2, 2]}[dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    _, u0, _ = W.config0(5, 2, K) if dim == 2 else (None, None, None)
    u = u0 if (dim == 2 and mesh.grid == [2 * K, 2 * K, 1]) else smooth_state(mesh, amp=0.5)
    # add a discontinuity so that the blended interface states are genuinely different
    g = mesh.grid
    u = u.copy()
    u[0][..., g[0] // 2:] *= 1.7
    u[dim + 1][..., g[0] // 2:] *= 1.3
    p = W.Params(mode=W.EXTERNAL)
    A = W.alpha_len(mesh, p)
    for trial in range(3):
        al = RNG.uniform(0.0, 1.0, size=(mesh.nel, A))
        d = O.rhs(mesh, p, u, alpha_in=al)
        tot = d.reshape(mesh.nvar, -1).sum(1)
        scale = np.abs(d).reshape(mesh.nvar, -1).sum(1)
        assert np.all(np.abs(tot) <= 1e-13 * scale), (tot, scale)
    # adaptive mode as well
    d = O.rhs(mesh, W.Params(), u)
    tot = d.reshape(mesh.nvar, -1).sum(1)
    assert np.all(np.abs(tot) <= 1e-13 * np.abs(d).reshape(mesh.nvar, -1).sum(1))


@pytest.mark.parametrize("dim,K", [(2, 4), (2, 8), (3, 4)])
def test_free_stream(dim, K):
    """A uniform state is preserved for any blending factors."""
    ne = {2: [3, 2], 3: [2, 2, 2]}[dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    u = np.zeros(mesh.shape())
    u[0], u[1], u[dim + 1] = 1.3, 0.4, 3.0
    if dim > 1:
        u[2] = -0.25
    p = W.Params(mode=W.EXTERNAL)
    A = W.alpha_len(mesh, p)
    al = RNG.uniform(0.0, 1.0, size=(mesh.nel, A))
    d = O.rhs(mesh, p, u, alpha_in=al)
    scale = 10.0 * K * max(ne)
    assert np.abs(d).max() <= 1e-13 * scale


@pytest.mark.parametrize("dim,K", [(1, 8), (2, 4), (2, 8), (3, 4)])
def test_free_stream_outflow(dim, K):
    """R16 (outflow as zero gradient of the subcell means): a uniform moving state on a mesh
    with outflow boundaries on every axis is preserved for any blending factors, the
    boundary faces included (the exterior state is the boundary cell's mean, equal to the
    interior one, so the common flux there is the physical flux of the state); the
    earlier reading (exterior = the interior face state) gave the same here, so this pins
    the boundary faces' consistency, not the choice between the two."""
    ne = {1: [5], 2: [3, 2], 3: [2, 2, 2]}[dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [1] * dim)
    u = np.zeros(mesh.shape())
    u[0], u[1], u[dim + 1] = 1.3, 0.9, 3.0
    if dim > 1:
        u[2] = -0.25
    p = W.Params(mode=W.EXTERNAL)
    A = W.alpha_len(mesh, p)
    al = RNG.uniform(0.0, 1.0, size=(mesh.nel, A))
    d = O.rhs(mesh, p, u, alpha_in=al)
    scale = 10.0 * K * max(ne)
    assert np.abs(d).max() <= 1e-13 * scale


def test_outflow_supersonic_exit_flux():
    """R16: at an outflow face of a supersonic exit the common flux is the physical flux
    of the boundary cell's mean (HLL upwinding of equal states), so for a state that is
    uniform except in the interior the boundary cell's update only sees its interior face:
    the change of bulk equals the difference of the physical fluxes at the two ends."""
    K, ne = 8, [4]
    mesh = W.Mesh(1, K, ne, [0.0], [1.0], [1])
    x = 0.5 * (mesh.edges(0)[1:] + mesh.edges(0)[:-1])
    rho = 1.0 + 0.2 * np.exp(-((x - 0.5) / 0.08) ** 2)
    v, pr = 3.0, 1.0                      # Mach > 2.5 everywhere: supersonic to the right
    u = np.zeros(mesh.shape())
    u[0, 0, 0] = rho
    u[1, 0, 0] = rho * v
    u[2, 0, 0] = pr / 0.4 + 0.5 * rho * v * v
    p = W.Params(mode=W.FORCE_FV)         # first-order FV: fluxes at subcell faces only
    d = O.rhs(mesh, p, u)
    # total change = (F(left end) - F(right end)) / |domain| with F the physical flux of the
    # end cells' means (the outflow exterior state repeats the end cell)
    def flux(r):
        m = r * v
        E = pr / 0.4 + 0.5 * r * v * v
        return np.array([m, m * v + pr, v * (E + pr)])
    total = d[:, 0, 0, :].sum(axis=1) / (K * ne[0])
    expect = flux(rho[0]) - flux(rho[-1])
    assert np.allclose(total, expect, rtol=1e-12, atol=1e-12)


def _shock_profile(x):
    rho = np.where(x < 0.43, 1.0, 0.3) + 0.05 * np.sin(6 * np.pi * x)
    v = np.where(x < 0.43, 0.5, 0.1)
    p = np.where(x < 0.43, 1.0, 0.2)
    return rho, v, p


@pytest.mark.parametrize("K", [4, 8])
def test_2d_y_invariant_equals_1d(K):
    """Data constant in y: the 2-D adaptive scheme reduces to the 1-D scheme
    (blending factors, right-hand side; the y-momentum change vanishes)."""
    ne = 6
    m1 = W.Mesh(1, K, [ne], [0.0], [1.0], [1])
    x = 0.5 * (m1.edges(0)[1:] + m1.edges(0)[:-1])
    rho, v, pr = _shock_profile(x)
    u1 = np.zeros(m1.shape())
    u1[0, 0, 0], u1[1, 0, 0], u1[2, 0, 0] = rho, rho * v, pr / 0.4 + 0.5 * rho * v * v
    m2 = W.Mesh(2, K, [ne, 2], [0.0, 0.0], [1.0, 0.7], [1, 0])
    u2 = np.zeros(m2.shape())
    u2[0, 0] = rho
    u2[1, 0] = rho * v
    u2[3, 0] = pr / 0.4 + 0.5 * rho * v * v
    p = W.Params()
    d1, i1 = O.rhs(m1, p, u1, full=True)
    d2, i2 = O.rhs(m2, p, u2, full=True)
    # the level structure of the test data is non-trivial
    assert np.any((i1["alpha"] > 0) & (i1["alpha"] < 1)) or np.any(i1["alpha"][:, 0] == 0)
    # alpha: 2-D sub-element (sx, sy) equals the 1-D sub-element sx
    A1, A2 = i1["alpha"].shape[1], i2["alpha"].shape[1]
    lv = _alpha_levels_1d(K)
    o1 = o2 = 0
    for n in lv:
        ns = K // n
        a1 = i1["alpha"][:, o1:o1 + ns]
        a2 = i2["alpha"][:, o2:o2 + ns * ns].reshape(2, ne, ns, ns)
        for ey in range(2):
            for sy in range(ns):
                assert np.abs(a2[ey, :, sy, :] - a1).max() <= 1e-12
        o1 += ns
        o2 += ns * ns
    for ey in range(2 * K):
        for v1, v2 in [(0, 0), (1, 1), (2, 3)]:
            assert np.abs(d2[v2, 0, ey] - d1[v1, 0, 0]).max() <= 1e-11 * np.abs(d1[v1]).max()
    assert np.abs(d2[2]).max() <= 1e-12 * np.abs(d1).max()


def test_3d_z_invariant_equals_2d():
    K = 4
    m2 = W.Mesh(2, K, [3, 2], [0, 0], [1, 1], [1, 0])
    _, u2full, _ = W.config0(7, 2, K)
    u2 = np.zeros(m2.shape())
    x = 0.5 * (m2.edges(0)[1:] + m2.edges(0)[:-1])
    y = 0.5 * (m2.edges(1)[1:] + m2.edges(1)[:-1])
    Y, X = np.meshgrid(y, x, indexing="ij")
    rho = np.where(X < 0.5, 1.0, 0.5) * (1 + 0.1 * np.sin(2 * np.pi * Y))
    u2[0, 0] = rho
    u2[1, 0] = 0.3 * rho
    u2[2, 0] = -0.1 * rho
    u2[3, 0] = np.where(X < 0.5, 1.0, 0.3) / 0.4 + 0.5 * 0.1 * rho
    m3 = W.Mesh(3, K, [3, 2, 1], [0, 0, 0], [1, 1, 0.5], [1, 0, 0])
    u3 = np.zeros(m3.shape())
    for z in range(K):
        u3[0, z], u3[1, z], u3[2, z], u3[4, z] = u2[0, 0], u2[1, 0], u2[2, 0], u2[3, 0]
    p = W.Params()
    d2 = O.rhs(m2, p, u2)
    d3 = O.rhs(m3, p, u3)
    for z in range(K):
        for v2, v3 in [(0, 0), (1, 1), (2, 2), (3, 4)]:
            assert np.abs(d3[v3, z] - d2[v2, 0]).max() <= 1e-11 * np.abs(d2[v2]).max()
    assert np.abs(d3[3]).max() <= 1e-12 * np.abs(d2).max()


@pytest.mark.parametrize("K", [4, 8])
def test_transposition_symmetry(K):
    """Swapping x and y (and the momentum components) commutes with the scheme."""
    mesh = W.Mesh(2, K, [2, 2], [0, 0], [1, 1], [0, 0])
    _, u, _ = W.config0(11, 2, K)
    ut = np.zeros_like(u)
    ut[0, 0] = u[0, 0].T
    ut[1, 0] = u[2, 0].T
    ut[2, 0] = u[1, 0].T
    ut[3, 0] = u[3, 0].T
    p = W.Params()
    d, i = O.rhs(mesh, p, u, full=True)
    dt, it = O.rhs(mesh, p, ut, full=True)
    sw = {0: 0, 1: 2, 2: 1, 3: 3}
    for v in range(4):
        assert np.abs(dt[v, 0] - d[sw[v], 0].T).max() <= 1e-12 * np.abs(d[sw[v]]).max()


def test_indicator_closed_cases():
    """Linear data: all smoothness measures agree, alpha = 1 (pure top-level DG).
    A strong jump inside an element: alpha = 0 at the top level (Sec. 2.7)."""
    K = 8
    mesh = W.Mesh(2, K, [2, 2], [0, 0], [1, 1], [1, 1])
    g = mesh.grid
    x = 0.5 * (mesh.edges(0)[1:] + mesh.edges(0)[:-1])
    y = 0.5 * (mesh.edges(1)[1:] + mesh.edges(1)[:-1])
    Y, X = np.meshgrid(y, x, indexing="ij")
    u = np.zeros(mesh.shape())
    u[0, 0] = 1.0 + 0.2 * X + 0.1 * Y
    u[3, 0] = 2.5 + 0.3 * Y
    d, info = O.rhs(mesh, W.Params(), u, full=True)
    assert np.all(info["alpha"][:, 0] == 1.0) and np.all(info["alpha"][:, 1:] == 0.0)
    dg = O.rhs(mesh, W.Params(mode=W.FORCE_DG), u)
    assert np.array_equal(d, dg)
    # a jump at x = 0.3 (inside element 0 of each row)
    u[0, 0] = np.where(X < 0.3, 1.0, 0.125)
    u[3, 0] = np.where(X < 0.3, 1.0, 0.1) / 0.4
    d, info = O.rhs(mesh, W.Params(), u, full=True)
    al = info["alpha"].reshape(2, 2, -1)
    assert np.all(al[:, 0, 0] == 0.0)      # elements holding the jump: top level rejected
    assert np.all(al[:, 1, 0] == 1.0)      # constant elements: pure top-level DG


def _squeeze_points(u, e, K, b, T):
    ub = u[:, 0, 0, e * K:(e + 1) * K]
    mean = ub.mean(axis=1, keepdims=True)
    ut = ub @ T["R"].T
    us = (1 - b) * mean + b * ut
    pts = np.concatenate([us, (us @ T["bm"])[:, None], (us @ T["bp"])[:, None]], axis=1)
    return pts, us, mean


def test_squeeze_pressure_binding():
    """Pressure dip at rest (p linear in the state): beta (eq. calc-squeezing-parameter)
    makes the whole check set permissible, keeps the mean, and is the largest such
    value: the binding point sits at p = epsilon (Sec. 2.4); independent tables."""
    K = 4
    mesh = W.Mesh(1, K, [3], [0.0], [1.0], [1])
    u = np.zeros(mesh.shape())
    pr = np.array([1, 1, 1e-4, 1, 1, 1, 1, 1, 1, 1, 1, 1.0])
    u[0, 0, 0], u[2, 0, 0] = 1.0, pr / 0.4
    _, info = O.rhs(mesh, W.Params(), u, full=True)
    beta = info["beta"]
    assert 0.0 < beta[0, 0] < 1.0 and beta[2, 0] == 1.0
    T = refs.np_tables(K)
    pts, us, mean = _squeeze_points(u, 0, K, beta[0, 0], T)
    pp = refs.pressure(pts, 1)
    # the squeeze targets p = epsilon = 1e-20 at the binding point: in floating point that
    # point lands within rounding of zero, every other point is strictly permissible
    assert np.all(pts[0] > 0) and pp.min() > -1e-15 * pp.max()
    assert abs(pp.min()) < 1e-12 and np.sort(pp)[1] > 1e-6
    assert np.abs(us @ T["w"] - mean[:, 0]).max() < 1e-14 * np.abs(mean).max() * 10


def test_squeeze_nonpositive_density_reading():
    """A reconstruction with rho <= 0 at a check point has p := -inf, so beta = 0 and
    the squeezed data is the (permissible) sub-element mean."""
    K = 4
    mesh = W.Mesh(1, K, [3], [0.0], [1.0], [1])
    u = np.zeros(mesh.shape())
    rho = np.array([1, 1, 1, 1e-3, 1, 1, 1, 1, 1, 1, 1, 1.0])
    u[0, 0, 0], u[2, 0, 0] = rho, 1.0 / 0.4
    _, info = O.rhs(mesh, W.Params(), u, full=True)
    T = refs.np_tables(K)
    pts, _, _ = _squeeze_points(u, 0, K, 1.0, T)
    assert pts[0].min() <= 0.0
    assert info["beta"][0, 0] == 0.0
    assert info["alpha"][0, 0] == 0.0


def test_adaptive_equals_dg_on_resolved_smooth_data():
    mesh = W.Mesh(2, 8, [3, 3], [0, 0], [1, 1], [0, 0])
    u = W.density_wave(mesh)
    d, info = O.rhs(mesh, W.Params(), u, full=True)
    assert np.all(info["alpha"][:, 0] == 1.0)
    assert np.array_equal(d, O.rhs(mesh, W.Params(mode=W.FORCE_DG), u))


def _l2_err(mesh, u, T):
    ex = W.density_wave(mesh, t=T, vel=(0.1, 0.1, 0.1))
    return math.sqrt(np.mean((u[0] - ex[0]) ** 2))


@pytest.mark.parametrize("K,nes", [(4, (4, 8)), (8, (2, 4))])
def test_convergence_order_density_wave(K, nes):
    """Advected density wave (an exact Euler solution), pure DG: the L2 error of the
    density decays with order >= K - 0.5 (the paper's EOC tables show ~K)."""
    T, dt = 0.004, 1e-4
    errs = []
    for ne in nes:
        mesh = W.Mesh(2, K, [ne, ne], [0, 0], [1, 1], [0, 0])
        u0 = W.density_wave(mesh)
        u, _ = O.rk3(mesh, W.Params(mode=W.FORCE_DG), u0, int(round(T / dt)), dt)
        errs.append(_l2_err(mesh, u, T))
    eoc = math.log(errs[0] / errs[1]) / math.log(nes[1] / nes[0])
    assert eoc >= K - 0.5, (errs, eoc)


def test_rk3_third_order_in_time():
    """Three-stage SSP-RK: halving dt divides the temporal error by ~8."""
    K = 8
    mesh = W.Mesh(1, K, [4], [0.0], [1.0], [0])
    u0 = W.density_wave(mesh, vel=(0.5, 0, 0), amp=0.3)
    p = W.Params(mode=W.FORCE_DG)
    T = 0.08
    ref, _ = O.rk3(mesh, p, u0, 640, T / 640)
    e = []
    for nst in (20, 40):
        u, _ = O.rk3(mesh, p, u0, nst, T / nst)
        e.append(np.abs(u - ref).max())
    rate = math.log2(e[0] / e[1])
    assert 2.7 < rate < 3.3, (e, rate)


def test_cfl_step():
    """dt = CFL dx / (2^(d-1) (2K-1) lambda_max) with lambda = max |v_a| + c over the means."""
    mesh, u, _ = W.config0(0, 16, 4)
    p = W.Params(cfl=0.5)
    rho, mx, my, E = u[0, 0], u[1, 0], u[2, 0], u[3, 0]
    pr = 0.4 * (E - 0.5 * (mx ** 2 + my ** 2) / rho)
    c = np.sqrt(1.4 * pr / rho)
    lam = max((np.abs(mx / rho) + c).max(), (np.abs(my / rho) + c).max())
    assert abs(O.max_dt(mesh, p, u) - 0.5 * (1 / 16) / (2 * 7 * lam)) < 1e-16


def test_nonpermissible_state_rejected():
    mesh, u, _ = W.config0(0, 2, 4)
    u = u.copy()
    u[0, 0, 3, 3] = -1.0
    with pytest.raises(O.OracleError):
        O.rhs(mesh, W.Params(), u)
