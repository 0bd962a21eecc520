"""The conservation stress test of Sec. 3.3 on the oracle: blending factors drawn at
random for every right-hand side (RANDOM mode) from SplitMix64, whose definition is
pinned here by its published reference outputs; the change of bulk (eq.
change-of-bulk) of every stage stays at round-off; the weighted blending factor of eq.
order-estimate against the weights of eq. blending-weights."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03338_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64_seed1234567.txt")
M64 = (1 << 64) - 1


def splitmix64(seed, k):
    """k-th output of SplitMix64 seeded with seed: the output function applied to
    seed + (k + 1) * 0x9e3779b97f4a7c15 (mod 2^64)."""
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def random_factors(seed, draw, nel, A):
    out = np.empty((nel, A))
    for e in range(nel):
        for q in range(A):
            out[e, q] = (splitmix64(seed, (draw * nel + e) * A + q) >> 11) * 2.0 ** -53
    return out


def test_splitmix64_reference_outputs():
    ref = [int(x) for x in open(GOLDEN).read().split("\n") if x and not x.startswith("#")]
    assert [splitmix64(1234567, k) for k in range(len(ref))] == ref


@pytest.mark.parametrize("dim,K", [(2, 4), (2, 8), (3, 4)])
def test_random_mode_draws_the_generator(dim, K):
    ne = [3, 2, 2][:dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    u = W.density_wave(mesh)
    p = W.Params(mode=W.RANDOM, seed=987654321)
    A = W.alpha_len(mesh, p)
    for draw in (0, 5):
        _, info = O.rhs(mesh, p, u, full=True, draw=draw)
        assert np.array_equal(info["alpha"], random_factors(p.seed, draw, mesh.nel, A))
    # with the drawn factors given, RANDOM equals EXTERNAL bit for bit
    d_r = O.rhs(mesh, p, u, draw=3)
    d_e = O.rhs(mesh, W.Params(mode=W.EXTERNAL), u, alpha_in=random_factors(p.seed, 3, mesh.nel, A))
    assert np.array_equal(d_r, d_e)


def _stress_state(mesh, seed=0):
    rng = np.random.default_rng(seed)
    u = W.density_wave(mesh, vel=(0.3, -0.2, 0.1), amp=0.3)
    u[mesh.dim + 1] *= 1.0 + 0.2 * rng.uniform(size=u[0].shape)
    return u


@pytest.mark.parametrize("dim,K,ne,steps", [(2, 4, [8, 8], 100), (2, 8, [4, 4], 30), (3, 4, [3, 3, 3], 10)])
def test_conservation_random_factors_every_stage(dim, K, ne, steps):
    """Sec. 3.3: factors drawn afresh for every stage, periodic mesh.  At every stage the
    change of bulk (eq. change-of-bulk, |Omega_q| as weight) vanishes to round-off
    against the sum of |d(u)/dt|; the stages, written out here, reproduce the oracle's
    own RANDOM-mode SSP-RK3 bit for bit (same draws in the same order)."""
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    p = W.Params(mode=W.RANDOM, seed=11)
    u = _stress_state(mesh)
    u0 = u.copy()
    vol = np.prod([1.0 / (n * K) for n in ne])
    draw, worst = 0, 0.0
    for _ in range(steps):
        dt = O.max_dt(mesh, p, u)
        stages = []
        L = O.rhs(mesh, p, u, draw=draw)
        stages.append(L)
        u1 = u + dt * L
        L = O.rhs(mesh, p, u1, draw=draw + 1)
        stages.append(L)
        u2 = 0.75 * u + 0.25 * (u1 + dt * L)
        L = O.rhs(mesh, p, u2, draw=draw + 2)
        stages.append(L)
        u_next = (1.0 / 3.0) * u + (2.0 / 3.0) * (u2 + dt * L)
        ref, _ = O.rk3(mesh, p, u, 1, dt_fixed=dt, draw=draw)
        assert np.array_equal(ref, u_next)
        for L in stages:
            bulk = vol * L.reshape(mesh.nvar, -1).sum(axis=1)
            scale = vol * np.abs(L).reshape(mesh.nvar, -1).sum(axis=1)
            worst = max(worst, float((np.abs(bulk) / scale).max()))
        u, draw = u_next, draw + 3
    assert worst <= 1e-13, worst
    # the domain totals of the state stay at their initial values
    tot0 = u0.reshape(mesh.nvar, -1).sum(axis=1)
    tot = u.reshape(mesh.nvar, -1).sum(axis=1)
    assert np.all(np.abs(tot - tot0) <= 1e-13 * np.abs(u0).reshape(mesh.nvar, -1).sum(axis=1))


@pytest.mark.parametrize("dim,K,top", [(2, 8, 0), (2, 4, 0), (3, 4, 0), (2, 8, 4)])
def test_alpha_bar_is_the_weighted_order(dim, K, top):
    """eq. order-estimate equals sum_n n theta^(n) with the product weights of eq.
    blending-weights (theta_FV carrying order 1), lies in [1, top]; 1 for pure FV and
    top for pure top-level DG."""
    ne = [3, 2, 2][:dim]
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    p = W.Params(top_level=top)
    A = W.alpha_len(mesh, p)
    levels = []
    n = top or K
    while n >= 2:
        levels.append(n)
        n //= 2
    al = np.random.default_rng(4).uniform(size=(mesh.nel, A))
    ab = O.alpha_bar(mesh, p, al)
    g = mesh.grid
    exp = np.zeros((g[2], g[1], g[0]))
    for e in range(mesh.nel):
        ex, ey, ez = e % ne[0], (e // ne[0]) % (ne[1] if dim > 1 else 1), e // (ne[0] * (ne[1] if dim > 1 else 1))
        for k in range(K if dim > 2 else 1):
            for j in range(K if dim > 1 else 1):
                for i in range(K):
                    prod, tot, off = 1.0, 0.0, 0
                    for n in levels:
                        ns = K // n
                        s = i // n + ns * ((j // n) + ns * (k // n))
                        a = al[e, off + s]
                        tot += n * a * prod
                        prod *= 1.0 - a
                        off += ns ** dim
                    tot += 1.0 * prod
                    exp[ez * K + k if dim > 2 else 0, ey * K + j if dim > 1 else 0, ex * K + i] = tot
    assert np.abs(ab - exp).max() <= 1e-14 * (top or K)
    assert ab.min() >= 1.0 and ab.max() <= (top or K)
    assert np.all(O.alpha_bar(mesh, p, np.zeros_like(al)) == 1.0)
    one_top = np.zeros_like(al)
    one_top[:, :(K // (top or K)) ** dim] = 1.0
    assert np.all(O.alpha_bar(mesh, p, one_top) == (top or K))
