"""The five-stage fourth-order SSP Runge-Kutta scheme the paper integrates with (Sec. 3;
Spiteri & Ruuth, SIAM J. Numer. Anal. 40 (2002)): its published Shu-Osher coefficients
pinned by the eight order conditions of a fourth-order method and by non-negativity
(the SSP property, coefficient 1.508), and the oracle's implementation pinned by its
fourth order in time on a smooth Euler flow."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03338_amd import workloads as W

# Shu-Osher form u_i = sum_j alpha_ij u_j + beta_ij dt L(u_j), as published
ALPHA = {(1, 0): 1.0,
         (2, 0): 0.444370493651235, (2, 1): 0.555629506348765,
         (3, 0): 0.620101851488403, (3, 2): 0.379898148511597,
         (4, 0): 0.178079954393132, (4, 3): 0.821920045606868,
         (5, 2): 0.517231671970585, (5, 3): 0.096059710526147, (5, 4): 0.386708617503269}
BETA = {(1, 0): 0.391752226571890, (2, 1): 0.368410593050371, (3, 2): 0.251891774271694,
        (4, 3): 0.544974750228521, (5, 3): 0.063692468666290, (5, 4): 0.226007483236906}


def butcher():
    """(A, b, c) of the Shu-Osher form: u_i = u^n + dt sum_j a_ij L(u_j)."""
    rows = np.zeros((6, 5))
    for i in range(1, 6):
        for j in range(i):
            rows[i] += ALPHA.get((i, j), 0.0) * rows[j]
            rows[i, j] += BETA.get((i, j), 0.0)
    A = rows[:5]
    return A, rows[5], A.sum(axis=1)


def test_coefficients_fourth_order_and_ssp():
    for i in range(1, 6):
        assert abs(sum(ALPHA.get((i, j), 0.0) for j in range(i)) - 1.0) < 1e-14   # consistency
    assert all(v >= 0.0 for v in ALPHA.values()) and all(v >= 0.0 for v in BETA.values())
    A, b, c = butcher()
    conds = [b.sum() - 1, b @ c - 1 / 2, b @ c ** 2 - 1 / 3, b @ A @ c - 1 / 6, b @ c ** 3 - 1 / 4,
             b @ (c * (A @ c)) - 1 / 8, b @ A @ c ** 2 - 1 / 12, b @ A @ A @ c - 1 / 24]
    assert max(abs(x) for x in conds) < 5e-15, conds
    ssp = min(ALPHA[k] / BETA[k] for k in BETA)
    assert abs(ssp - 1.508) < 1e-3
    # stability polynomial: 1 + z + z^2/2 + z^3/6 + z^4/24 + g5 z^5 (fifth coefficient free)
    e = np.ones(5)
    coef = [1.0, b @ e, b @ A @ e, b @ A @ A @ e, b @ A @ A @ A @ e]
    assert np.allclose(coef, [1, 1, 1 / 2, 1 / 6, 1 / 24], rtol=0, atol=1e-14)


def test_oracle_rk54_fourth_order_in_time():
    """The density wave (an exact Euler solution) on a fixed mesh in pure DG mode, to
    T = 0.1 against 1024 steps of the same scheme: SSP-RK(5,4) errors fall by 2^4 from 8 to
    16 steps (below that the reference's own rounding, ~2e-12, is reached); SSP-RK3 falls
    by 2^3 from 16 to 64 steps (8 steps exceed its stability limit)."""
    mesh = W.Mesh(1, 8, [4], [0.0], [1.0], [0])
    u0 = W.density_wave(mesh, vel=(0.5, 0, 0), amp=0.1)
    T = 0.1

    def errs(integ, ns):
        p = W.Params(mode=W.FORCE_DG, integrator=integ)
        ref, _ = O.rk3(mesh, p, u0, 1024, dt_fixed=T / 1024)
        return [np.abs(O.rk3(mesh, p, u0, n, dt_fixed=T / n)[0] - ref).max() for n in ns]

    e4 = errs(1, (8, 16))
    assert np.log2(e4[0] / e4[1]) > 3.7, e4
    e3 = errs(0, (16, 32, 64))
    rates3 = [np.log2(e3[i] / e3[i + 1]) for i in range(2)]
    assert all(2.8 < r < 3.3 for r in rates3), rates3


def test_oracle_rk54_step_is_the_shu_osher_form():
    """Two adaptive SSP-RK(5,4) steps of the oracle equal the Shu-Osher form above composed
    from the oracle's right-hand sides (to rounding)."""
    mesh, u0, _ = W.config0(1, 6, 4)
    p = W.Params(integrator=1)
    dt = 0.8 * O.max_dt(mesh, p, u0)
    got, _ = O.rk3(mesh, p, u0, 2, dt_fixed=dt)
    u = u0.copy()
    for _ in range(2):
        st, Ls = {0: u}, {}
        for i in range(1, 6):
            Ls[i - 1] = O.rhs(mesh, p, st[i - 1])
            acc = 0.0
            for j in range(i):
                acc = acc + ALPHA.get((i, j), 0.0) * st[j] + BETA.get((i, j), 0.0) * dt * Ls.get(j, 0.0)
            st[i] = acc
        u = st[5]
    assert np.abs(got - u).max() <= 1e-13 * np.abs(u).max()


def test_oracle_rk54_random_draws_per_stage():
    """Five right-hand sides per step draw five factor sets: two steps equal ten random
    right-hand sides composed by hand in the Shu-Osher form."""
    mesh = W.Mesh(2, 4, [3, 3], [0, 0], [1, 1], [0, 0])
    u0 = W.density_wave(mesh, vel=(0.3, -0.2, 0), amp=0.2)
    p = W.Params(mode=W.RANDOM, seed=5, integrator=1)
    dt = 0.5 * O.max_dt(mesh, p, u0)
    got, _ = O.rk3(mesh, p, u0, 2, dt_fixed=dt)
    u, d = u0.copy(), 0
    for _ in range(2):
        st = {0: u}
        Ls = {}
        for i in range(1, 6):
            j_last = i - 1
            Ls[j_last] = O.rhs(mesh, p, st[j_last], draw=d)
            d += 1
            acc = 0.0
            for j in range(i):
                acc = acc + ALPHA.get((i, j), 0.0) * st[j] + BETA.get((i, j), 0.0) * dt * Ls.get(j, 0.0)
            st[i] = acc
        u = st[5]
    assert np.abs(got - u).max() <= 1e-13 * np.abs(u).max()
