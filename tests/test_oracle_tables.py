"""Pins of the oracle's operator tables (Sec. 2.1-2.4, 2.6) against closed forms,
the identities the paper proves, and an independent numpy construction."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.refs import np_tables

LEVELS = [2, 4, 8]


@pytest.mark.parametrize("n", LEVELS)
@pytest.mark.parametrize("fam", [0, 1])
def test_identities(n, fam):
    t = O.tables(n, fam)
    one = np.ones(n)
    tol = 8 * n * np.finfo(float).eps
    # weights sum to one on [-1/2, 1/2]
    assert abs(t["w"].sum() - 1.0) < tol
    # w^T D = 0 (eq. dg-vol-mat-property) and Dcal 1 = 0
    assert np.abs(t["w"] @ t["D"]).max() < tol * np.abs(t["D"]).max()
    assert np.abs(t["Dcal"] @ one).max() < tol * np.abs(t["Dcal"]).max()
    # 1^T P = n w^T (eq. projection-mat-property)
    assert np.abs(one @ t["P"] - n * t["w"]).max() < tol
    # P R = I and w^T R = 1^T / n (eq. reconstruction-mat-property)
    assert np.abs(t["P"] @ t["R"] - np.eye(n)).max() < tol * np.abs(t["R"]).max()
    assert np.abs(t["w"] @ t["R"] - one / n).max() < tol * np.abs(t["R"]).max()
    # sum_i l_i(+-1/2) = 1 and w^T B^(0) = 1^T Delta^(S) = (-1, 0, ..., 0, 1)
    assert abs(t["bm"].sum() - 1) < tol and abs(t["bp"].sum() - 1) < tol
    # 1^T Bhat = n (w^T B^(0)): first column sums to -n, last to +n
    assert abs(t["Bhl"].sum() + n) < tol * n * 10 and abs(t["Bhr"].sum() - n) < tol * n * 10
    # 1^T Dhat = n w^T D = 0
    assert np.abs(one @ t["Dhat"]).max() < tol * np.abs(t["Dhat"]).max() * n
    # interface interpolation: rows sum to one; last row of I+ is b+, first row of I- is b-
    assert np.abs(t["Ip"].sum(1) - 1).max() < tol * 10 and np.abs(t["Im"].sum(1) - 1).max() < tol * 10
    assert np.abs(t["Ip"][-1] - t["bp"]).max() < tol and np.abs(t["Im"][0] - t["bm"]).max() < tol
    # consecutive subcell interfaces coincide: I+ row i == I- row i+1
    assert np.abs(t["Ip"][:-1] - t["Im"][1:]).max() < tol * 10


def test_closed_forms_n2():
    """n = 2: Gauss nodes +-1/(2 sqrt 3) give P = [[1/2+sqrt3/4, 1/2-sqrt3/4], ...] and
    R = [[1/2+1/sqrt3, 1/2-1/sqrt3], ...]; Lobatto nodes +-1/2 give P = [[3/4,1/4],[1/4,3/4]]
    and R = [[3/2,-1/2],[-1/2,3/2]] (subcell means of the linear interpolant)."""
    t = O.tables(2, 0)
    a, b = 0.5 + math.sqrt(3) / 4, 0.5 - math.sqrt(3) / 4
    assert np.allclose(t["P"], [[a, b], [b, a]], rtol=0, atol=2e-16)
    c, d = 0.5 + 1 / math.sqrt(3), 0.5 - 1 / math.sqrt(3)
    assert np.allclose(t["R"], [[c, d], [d, c]], rtol=0, atol=4e-16)
    assert np.allclose(t["xi"], [-0.5 / math.sqrt(3), 0.5 / math.sqrt(3)], rtol=0, atol=1e-16)
    t = O.tables(2, 1)
    assert np.allclose(t["P"], [[0.75, 0.25], [0.25, 0.75]], rtol=0, atol=2e-16)
    assert np.allclose(t["R"], [[1.5, -0.5], [-0.5, 1.5]], rtol=0, atol=4e-16)
    # D for n = 2 is the same for both node sets up to the node spacing: D = [[-1,-1],[1,1]]/h
    t = O.tables(2, 0)
    h = 1 / math.sqrt(3)
    assert np.allclose(t["Dcal"], np.array([[-1, 1], [-1, 1]]) / h, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", LEVELS)
@pytest.mark.parametrize("fam", [0, 1])
def test_against_numpy_builder(n, fam):
    """A second, independent construction (numpy Gauss rule and polynomial algebra)."""
    t = O.tables(n, fam)
    r = np_tables(n, lobatto=bool(fam))
    for k_or, k_np in [("xi", "x"), ("w", "w"), ("Dcal", "Dcal"), ("D", "D"), ("P", "P"), ("R", "R"),
                       ("bm", "bm"), ("bp", "bp"), ("Ip", "Ip"), ("Im", "Im")]:
        scale = max(1.0, np.abs(r[k_np]).max())
        assert np.abs(t[k_or] - r[k_np]).max() < 1e-12 * scale, k_or
    Dhat = r["P"] @ r["D"]
    assert np.abs(t["Dhat"] - Dhat).max() < 1e-12 * np.abs(Dhat).max()


@pytest.mark.parametrize("n", LEVELS)
def test_reconstruction_exact_for_polynomials(n):
    """Means of any polynomial of degree < n are mapped by R to its nodal values (Sec. 2.4)."""
    t = O.tables(n, 0)
    for deg in range(n):
        # exact subcell means of x^deg on [-1/2, 1/2] split in n subcells
        edges = -0.5 + np.arange(n + 1) / n
        means = n * (edges[1:] ** (deg + 1) - edges[:-1] ** (deg + 1)) / (deg + 1)
        nodal = t["R"] @ means
        assert np.abs(nodal - t["xi"] ** deg).max() < 1e-13


def test_gauss_golden():
    """Tabulated Gauss-Legendre nodes on [-1,1] (tests/golden/gauss_nodes.txt, standard
    published values to 16 digits) mapped to [-1/2, 1/2]."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "gauss_nodes.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for r in rows:
        n = int(r[0])
        xs = np.array(sorted(float(v) for v in r[1:]))
        t = O.tables(n, 0)
        assert np.abs(t["xi"] - 0.5 * xs).max() < 1e-15
