"""CPU-side checks of the library: it loads, exports every entry point the
header declares, and its independent table builder agrees with the oracle's."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03338_amd import sedg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(sedg_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = sedg.load()
    decl = _declared()
    assert "sedg_rhs" in decl and "sedg_rk_step" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert set(sedg.EXPORTED) <= set(decl)


def test_strerror():
    assert sedg.strerror(0) == "ok"
    assert "non-permissible" in sedg.strerror(-4)


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("fam", [0, 1])
def test_two_table_builders_agree(n, fam):
    """The library (quad precision, barycentric derivative, monomial integration) and
    the oracle (long double, product-rule derivative, Gauss quadrature) build the
    same operators to within 4 ulp of the table's scale."""
    a, b = O.tables(n, fam), sedg.tables(n, fam)
    for k in a:
        scale = np.abs(a[k]).max()
        tol = 4 * np.spacing(np.maximum(np.abs(a[k]), 1e-3 * scale))
        assert np.all(np.abs(a[k] - b[k]) <= tol), k


def test_bad_level_rejected():
    with pytest.raises(sedg.SedgError):
        sedg.tables(3, 0)


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("fam", [0, 1])
def test_two_nc_table_builders_agree(n, fam):
    """Refinement, coarsening and mortar tables: library (quad precision) against the
    oracle (long double), built independently."""
    a, b = sedg.nc_tables(n, fam), O.nc_tables(n, fam)
    for k in ("Z", "Q", "Lm", "Lp"):
        assert np.abs(a[k] - b[k]).max() <= 8 * np.finfo(float).eps * max(1.0, np.abs(b[k]).max()), k


@pytest.mark.parametrize("case", ["no_elements", "empty_box", "bad_bc", "gamma", "family", "dim", "K",
                                  "too_many_elements", "axis_subcells_overflow", "element_count_overflow"])
def test_create_rejects_bad_meshes_before_any_device_work(case):
    """sedg_create validates the mesh before it touches the device (so these run on the
    CPU): no elements along an axis, an empty box, an unknown boundary condition, gamma
    <= 1, an unknown node family, more than SEDG_MAX_ELEMENTS = 2^28 - 1 elements, more
    than INT_MAX subcells along an axis, or an element count beyond 32 bits (which would
    wrap in 32-bit arithmetic) give SEDG_EINVAL, an unsupported dimension or K
    SEDG_EUNSUPPORTED."""
    from paper_2011_03338_amd import workloads as W
    mesh = dict(dim=2, K=8, nelem=[4, 4], lo=[0.0, 0.0], hi=[1.0, 1.0], bc=[0, 0])
    expect = sedg.SEDG_EINVAL
    if case == "no_elements":
        mesh["nelem"] = [4, 0]
    elif case == "empty_box":
        mesh["hi"] = [1.0, 0.0]
    elif case == "bad_bc":
        mesh["bc"] = [0, 7]
    elif case == "dim":
        mesh.update(dim=1, nelem=[4], lo=[0.0], hi=[1.0], bc=[0])
        expect = sedg.SEDG_EUNSUPPORTED
    elif case == "K":
        mesh["K"] = 6
        expect = sedg.SEDG_EUNSUPPORTED
    elif case == "too_many_elements":
        mesh["nelem"] = [16384, 16384]          # 2^28 elements, one above the limit
    elif case == "axis_subcells_overflow":
        mesh["nelem"] = [(2 ** 31 - 1) // 8 + 1, 1]
    elif case == "element_count_overflow":
        # 2^32 + 2^16 elements: the product wraps to 65536 in 32-bit arithmetic
        mesh["nelem"] = [65537, 65536]
    m = W.Mesh(mesh["dim"], mesh["K"], mesh["nelem"], mesh["lo"], mesh["hi"], mesh["bc"],
               gamma=1.0 if case == "gamma" else 1.4, family=5 if case == "family" else 0)
    with pytest.raises(sedg.SedgError) as ei:
        sedg.Solver(m, W.Params())
    assert ei.value.code == expect


@pytest.mark.parametrize("nelem", [[16384, 16384], [65537, 65536], [(2 ** 31 - 1) // 8 + 1, 1]])
def test_batch_and_noalloc_reject_oversized_meshes_before_any_device_work(nelem):
    """sedg_batch_create (per member) and sedg_rhs_noalloc apply the same mesh limits as
    sedg_create and return SEDG_EINVAL before any device work or use of the state
    pointers (the pointers passed here are never dereferenced)."""
    import ctypes
    from paper_2011_03338_amd import workloads as W
    lib = sedg.load()
    ok = W.Mesh(2, 8, [4, 4], [0.0, 0.0], [1.0, 1.0], [0, 0])
    big = W.Mesh(2, 8, nelem, [0.0, 0.0], [1.0, 1.0], [0, 0])
    p = sedg.params_c(W.Params())
    arr = (sedg.Mesh_c * 2)(sedg.mesh_c(ok), sedg.mesh_c(big))
    h = ctypes.c_void_p()
    assert lib.sedg_batch_create(arr, 2, ctypes.byref(p), ctypes.byref(h)) == sedg.SEDG_EINVAL
    assert not h.value
    rc = lib.sedg_rhs_noalloc(ctypes.byref(sedg.mesh_c(big)), ctypes.byref(p), ctypes.c_void_p(16),
                              ctypes.c_void_p(32), None, None)
    assert rc == sedg.SEDG_EINVAL
