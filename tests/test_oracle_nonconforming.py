"""Pins of the non-conforming building blocks of the appendix (4:1 interfaces): the
expansion E, compression C, projections Z = P^(n->2n), Q = P^(n->n/2) and the mortar
matrices L_+-, and the blended refinement (eq. 3D-refinement) and coarsening (eq.
3D-coarsening) of the oracle, against what the definitions fix: conservation of every
element's integral for any factors, exactness on polynomial data, the pure-FV limits
(E and C: piecewise-constant copies and averages), and the single-level formula written
out with numpy tables."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npp

from oracle import oracle as O
from paper_2011_03338_amd import workloads as W
from tests import refs


def _means_of_poly(coef, edges):
    F = npp.polyint(coef)
    return (npp.polyval(edges[1:], F) - npp.polyval(edges[:-1], F)) / np.diff(edges)


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("fam", [0, 1])
def test_projection_tables(n, fam):
    T = O.nc_tables(n, fam)
    t = refs.np_tables(n, lobatto=bool(fam))
    Z, Q = T["Z"], T["Q"]
    # partition of unity and the mean: 1^T Z = 2n w^T, 1^T Q = (n/2) w^T (as 1^T P = n w^T)
    assert np.allclose(Z.sum(axis=1), 1.0, atol=1e-14) and np.allclose(Q.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(Z.sum(axis=0), 2 * n * t["w"], atol=1e-13)
    assert np.allclose(Q.sum(axis=0), (n / 2) * t["w"], atol=1e-13)
    # exact on polynomials of degree < n: nodal values -> exact subcell means
    rng = np.random.default_rng(n + 10 * fam)
    coef = rng.standard_normal(n)
    nod = npp.polyval(t["x"], coef)
    assert np.allclose(Z @ nod, _means_of_poly(coef, np.linspace(-0.5, 0.5, 2 * n + 1)), atol=1e-12)
    assert np.allclose(Q @ nod, _means_of_poly(coef, np.linspace(-0.5, 0.5, n // 2 + 1)), atol=1e-12)
    # integral additivity: averaging pairs of the 2n means gives P, pairs of P's n means Q
    C2 = 0.5 * np.kron(np.eye(n), np.ones((1, 2)))
    assert np.allclose(C2 @ Z, t["P"], atol=1e-13)
    if n >= 2:
        C1 = 0.5 * np.kron(np.eye(n // 2), np.ones((1, 2)))
        assert np.allclose(C1 @ t["P"], Q, atol=1e-13)


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("fam", [0, 1])
def test_mortar_matrices(n, fam):
    """The L2 projection back to the coarse face (quadrature on the collocation nodes) is
    exact for a coarse polynomial whose product with the basis the rule integrates
    exactly: its two halves, interpolated at the fine faces' nodes (x/2 -+ 1/4) and
    projected with L_-+, return it.  Gauss nodes (degree 2n - 1): every polynomial of
    degree < n, L_- I_- + L_+ I_+ = I.  LGL nodes (degree 2n - 3): degree < n - 1."""
    T = O.nc_tables(n, fam)
    t = refs.np_tables(n, lobatto=bool(fam))
    Im = np.array([[npp.polyval(0.5 * t["x"][k] - 0.25, t["basis"][j]) for j in range(n)] for k in range(n)])
    Ip = np.array([[npp.polyval(0.5 * t["x"][k] + 0.25, t["basis"][j]) for j in range(n)] for k in range(n)])
    M = T["Lm"] @ Im + T["Lp"] @ Ip
    if fam == 0:
        assert np.allclose(M, np.eye(n), atol=1e-12)
    deg = n - 1 if fam == 0 else n - 2
    coef = np.random.default_rng(n).standard_normal(deg + 1)
    nod = npp.polyval(t["x"], coef)
    assert np.allclose(M @ nod, nod, atol=1e-12)


def _mesh(dim, K, ne, fam=0, bc=0):
    return W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [bc] * dim, family=fam)


def _random_state(mesh, seed=0):
    rng = np.random.default_rng(seed)
    u = np.zeros(mesh.shape())
    u[0] = 1.0 + 0.5 * rng.uniform(size=u[0].shape)
    for a in range(mesh.dim):
        u[1 + a] = 0.2 * rng.standard_normal(u[0].shape)
    u[mesh.dim + 1] = 3.0 + rng.uniform(size=u[0].shape)
    return u


CASES = [(2, 4, [3, 2], 0), (2, 8, [2, 2], 0), (2, 8, [2, 1], 1), (3, 4, [2, 2, 1], 0)]


@pytest.mark.parametrize("dim,K,ne,fam", CASES)
def test_refine_coarsen_conserve(dim, K, ne, fam):
    """Every element's integral is kept by refinement and by coarsening, for random
    factors on every level."""
    mesh = _mesh(dim, K, ne, fam)
    p = W.Params()
    A = W.alpha_len(mesh, p)
    u = _random_state(mesh)
    al = np.random.default_rng(7).uniform(size=(mesh.nel, A))
    uf = O.refine(mesh, p, u, al)
    fm = O.fine_mesh(mesh)
    sums_c = u.reshape(mesh.nvar, -1).sum(axis=1)
    sums_f = uf.reshape(mesh.nvar, -1).sum(axis=1) / 2 ** dim
    assert np.allclose(sums_f, sums_c, rtol=1e-13, atol=0)
    alf = np.random.default_rng(8).uniform(size=(fm.nel, A))
    uc = O.coarsen(mesh, p, uf, alf)
    assert np.allclose(uc.reshape(mesh.nvar, -1).sum(axis=1), sums_c, rtol=1e-13, atol=0)


@pytest.mark.parametrize("dim,K,ne,fam", CASES)
def test_refine_coarsen_limits(dim, K, ne, fam):
    """Pure FV (all factors 0): refinement copies every mean into its 2^d children (E) and
    coarsening averages them back (C E = I), exactly.  Pure top-level DG on data that is
    a polynomial of degree < K per element: refinement gives the children's exact means,
    and coarsening those back gives the parents' exact means."""
    mesh = _mesh(dim, K, ne, fam)
    p = W.Params()
    A = W.alpha_len(mesh, p)
    fm = O.fine_mesh(mesh)
    u = _random_state(mesh)
    uf = O.refine(mesh, p, u, np.zeros((mesh.nel, A)))
    g = mesh.grid
    exp = u
    for a in range(dim):
        exp = np.repeat(exp, 2, axis=3 - a)
    assert np.array_equal(uf, exp)
    assert np.allclose(O.coarsen(mesh, p, uf, np.zeros((fm.nel, A))), u, rtol=0, atol=1e-15)
    # separable polynomial of degree K-1 per axis (one global polynomial is one per element)
    rng = np.random.default_rng(3)
    cx = [rng.standard_normal(K) * 0.1 for _ in range(dim)]
    top = np.zeros((mesh.nel, A))
    top[:, 0] = 1.0

    def poly_means(m):
        out = np.ones((1,) * 3)
        for a in range(dim):
            mm = _means_of_poly(cx[a], m.edges(a) * 2.0 - 1.0)
            shape = [1, 1, 1]
            shape[2 - a] = -1
            out = out * mm.reshape(shape)
        gg = m.grid
        return np.broadcast_to(1.0 + out, (gg[2], gg[1], gg[0]))

    uc = np.zeros(mesh.shape())
    for v in range(mesh.nvar):
        uc[v] = poly_means(mesh) * (1.0 + v)
    uf_exact = np.zeros(fm.shape())
    for v in range(mesh.nvar):
        uf_exact[v] = poly_means(fm) * (1.0 + v)
    got = O.refine(mesh, p, uc, top)
    assert np.abs(got - uf_exact).max() <= 1e-12 * np.abs(uf_exact).max()
    back = O.coarsen(mesh, p, uf_exact, np.tile(top[:1], (fm.nel, 1)))
    assert np.abs(back - uc).max() <= 1e-12 * np.abs(uc).max()


def test_refine_single_level_formula_2d():
    """eq. 3D-refinement as printed, in 2-D with numpy tables: r = (1 - a) u x_1 E x_2 E +
    a (u R^T R) x_1 Z x_2 Z per element, against the oracle with single-level factors
    (level mask {K}: factor a on the element, 0 below)."""
    K = 8
    mesh = _mesh(2, K, [2, 3])
    p = W.Params(level_mask=1 << 3)
    A = W.alpha_len(mesh, p)
    u = _random_state(mesh, 4)
    a_el = np.array([0.0, 0.3, 1.0, 0.65, 0.1, 0.9])
    al = np.zeros((mesh.nel, A))
    al[:, 0] = a_el
    got = O.refine(mesh, p, u, al)
    t = refs.np_tables(K)
    T = O.nc_tables(K)
    Z = T["Z"]
    E = np.kron(np.eye(K), np.ones((2, 1)))
    for e in range(mesh.nel):
        ex, ey = e % 2, e // 2
        for v in range(mesh.nvar):
            ub = u[v, 0, ey * K:(ey + 1) * K, ex * K:(ex + 1) * K]         # [y, x]
            nod = t["R"] @ ub @ t["R"].T
            r = (1 - a_el[e]) * (E @ ub @ E.T) + a_el[e] * (Z @ nod @ Z.T)
            blk = got[v, 0, 2 * ey * K:2 * (ey + 1) * K, 2 * ex * K:2 * (ex + 1) * K]
            assert np.abs(blk - r).max() <= 1e-12 * np.abs(r).max(), (e, v)
