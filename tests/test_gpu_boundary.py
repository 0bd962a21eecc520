"""GPU tests of the boundary's state, logging, random-factor and diagnostic entry
points, through the C ABI: sedg_init_state, the factor and step-size logs of
sedg_rk_step, SEDG_RANDOM mode against the oracle's RANDOM mode (the same generator on
both sides), the conservation stress test of Sec. 3.3 at every stage, sedg_diagnose
against the oracle (change of bulk, eq. order-estimate, activity counts), and the
frozen forward map sedg_rk_step_frozen."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_03338_amd import adjoint as ADJ, sedg, workloads as W
from tests.parity import DEV, RHS_TOL, STATE_TOL, blast_3d_k8, rel_err, say
from tests.test_oracle_random import random_factors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sedg.load()
    yield


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def test_init_state_copies_and_validates():
    mesh, u, _ = W.config0(0, 8, 4)
    s = sedg.Solver(mesh, W.Params())
    ug = torch.zeros(s.state_len, dtype=torch.float64, device=DEV)
    s.init_state(ug, u)
    assert np.array_equal(ug.cpu().numpy(), u.reshape(-1))
    bad = u.copy()
    bad[3, 0, 13, 9] = -5.0      # negative energy at subcell (9, 13): element 2 + 8 * 3
    bad[0, 0, 30, 31] = np.nan   # a later element
    with pytest.raises(sedg.SedgError) as ei:
        s.init_state(ug, bad)
    assert ei.value.code == sedg.SEDG_ESTATE and ei.value.element == 26
    s.check()                    # the flag was cleared
    s.close()


def test_step_logs_fixed_and_cfl():
    """dt_log receives the fixed step too; alpha_log receives every stage's factors, the
    same as the step tape records."""
    mesh, u, _ = W.config0(2, 6, 8)
    p = W.Params()
    s = sedg.Solver(mesh, p)
    A = s.alpha_len
    for dt_fixed in (1e-3, 0.0):
        ua = _t(u)
        dts = torch.full((4,), -1.0, dtype=torch.float64, device=DEV)
        alog = torch.full((4 * 3 * A,), -1.0, dtype=torch.float64, device=DEV)
        s.rk_step(ua, 4, dt_fixed, dts, alog)
        s.check()
        if dt_fixed > 0:
            assert torch.all(dts == dt_fixed)
        ub = _t(u)
        tape = torch.empty(s.tape_len, dtype=torch.float64, device=DEV)
        ns = s.state_len
        for j in range(4):
            s.rk_step_tape(ub, dts[j:j + 1], tape)
            fz = tape[3 * ns:3 * ns + 3 * A].view(3, A)
            assert torch.equal(alog.view(4, 3, A)[j], fz), j
        assert torch.equal(ua, ub)
    s.close()


@pytest.mark.parametrize("K,ne", [(4, 6), (8, 3)])
def test_random_rhs_matches_oracle(K, ne):
    """SEDG_RANDOM draws exactly the oracle's factors (bitwise), draw after draw, and the
    right-hand sides agree within 1e-12."""
    mesh, u, _ = W.config0(1, ne, K)
    p = W.Params(mode=W.RANDOM, seed=20240517)
    s = sedg.Solver(mesh, p)
    ug = _t(u)
    A = s.alpha_len
    for draw in range(3):
        d = torch.zeros_like(ug)
        al = torch.zeros(A, dtype=torch.float64, device=DEV)
        s.rhs(ug, d, al)
        s.check()
        d_o, info = O.rhs(mesh, p, u, full=True, draw=draw)
        assert np.array_equal(al.cpu().numpy().reshape(info["alpha"].shape), info["alpha"])
        err = rel_err(d.cpu().numpy(), d_o)
        say("  random rhs K=%d draw %d rel_err=%.3e" % (K, draw, err))
        assert err <= RHS_TOL
    # sedg_set_params restarts the draws
    s.set_params(p)
    al = torch.zeros(A, dtype=torch.float64, device=DEV)
    s.rhs(ug, torch.zeros_like(ug), al)
    assert np.array_equal(al.cpu().numpy().reshape(mesh.nel, -1), random_factors(p.seed, 0, mesh.nel, A // mesh.nel))
    s.close()


@pytest.mark.parametrize("K,ne", [(4, 16), (8, 8)])
def test_random_rk_steps_match_oracle(K, ne):
    """100 SSP-RK3 steps with factors drawn for every stage: state within 1e-9 of the
    oracle's RANDOM-mode steps, the logged factors the oracle's draws 0 .. 299."""
    mesh, u, _ = W.config0(0, ne, K)
    p = W.Params(mode=W.RANDOM, seed=7)
    u_o, dts_o = O.rk3(mesh, p, u, 100)
    s = sedg.Solver(mesh, p)
    A = s.alpha_len
    ug = _t(u)
    dts = torch.zeros(100, dtype=torch.float64, device=DEV)
    alog = torch.zeros(300 * A, dtype=torch.float64, device=DEV)
    s.rk_step(ug, 100, 0.0, dts, alog)
    s.check()
    err = rel_err(ug.cpu().numpy(), u_o)
    dterr = np.abs(dts.cpu().numpy() - dts_o).max() / dts_o.max()
    say("  random rk3 K=%d 100 steps rel_err=%.3e dt_err=%.3e" % (K, err, dterr))
    assert err <= STATE_TOL and dterr <= 1e-11
    la = alog.view(300, mesh.nel, A // mesh.nel).cpu().numpy()
    for d in (0, 1, 2, 150, 299):
        assert np.array_equal(la[d], random_factors(p.seed, d, mesh.nel, A // mesh.nel)), d
    s.close()


@pytest.mark.parametrize("dim,K,ne", [(2, 8, [16, 16]), (2, 4, [32, 24]), (3, 4, [6, 5, 4])])
def test_conservation_stress_every_stage(dim, K, ne):
    """Sec. 3.3 on the GPU: factors drawn at random for every stage on a periodic mesh,
    100 steps (20 in 3-D); every stage's right-hand side (the stage state and its factors
    from the step tape, evaluated again with those factors) has a change of bulk within
    1e-13 of its absolute bulk, and sedg_diagnose reports the same sums."""
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim)
    rng = np.random.default_rng(3)
    u = W.density_wave(mesh, vel=(0.3, -0.2, 0.1), amp=0.3)
    u[dim + 1] *= 1.0 + 0.2 * rng.uniform(size=u[0].shape)
    steps = 100 if dim == 2 else 20
    pr = W.Params(mode=W.RANDOM, seed=99)
    s = sedg.Solver(mesh, pr)
    se = sedg.Solver(mesh, W.Params(mode=W.EXTERNAL))
    A, ns = s.alpha_len, s.state_len
    ug = _t(u)
    tape = torch.empty(s.tape_len, dtype=torch.float64, device=DEV)
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    d = torch.zeros_like(ug)
    vol = float(np.prod([1.0 / (n * K) for n in ne]))
    worst = 0.0
    tot0 = ug.view(mesh.nvar, -1).sum(1)
    for j in range(steps):
        s.max_dt(ug, dt)
        s.rk_step_tape(ug, dt, tape)
        for k in range(3):
            uk = tape[k * ns:(k + 1) * ns]
            ak = tape[3 * ns + k * A:3 * ns + (k + 1) * A]
            se.rhs(uk.contiguous(), d, None, None, ak.contiguous())
            L = d.view(mesh.nvar, -1)
            bulk = (vol * L.sum(1)).abs()
            scale = vol * L.abs().sum(1)
            worst = max(worst, float((bulk / scale).max()))
    s.check()
    se.check()
    tot = ug.view(mesh.nvar, -1).sum(1)
    drift = float(((tot - tot0).abs() / ug.view(mesh.nvar, -1).abs().sum(1)).max())
    say("  stress %s: worst stage change of bulk %.3e of |bulk|, total drift %.3e" % (ne, worst, drift))
    assert worst <= 1e-13 and drift <= 1e-13
    # the library's own change-of-bulk diagnostic on a fresh draw at the final state
    dg = s.diagnose(ug, d)
    for v in range(mesh.nvar):
        sv = vol * float(d.view(mesh.nvar, -1)[v].sum())
        assert abs(dg["bulk_change"][v] - sv) <= 1e-12 * dg["bulk_abs"][v]
        assert abs(dg["bulk_change"][v]) <= 1e-13 * dg["bulk_abs"][v]
    s.close()
    se.close()


@pytest.mark.parametrize("case", ["sedov narrow", "config0 K8", "sedov K4", "3-D blast K8"])
def test_diagnose_matches_oracle(case):
    """sedg_diagnose against the oracle's analysis of the same state: fallback count
    (integer, exact), squeezed and rejected sub-elements, elements by lowest order
    carrying weight, and the weighted blending factor of every subcell (eq.
    order-estimate, from the oracle's factors)."""
    mesh, u = {"sedov narrow": lambda: W.sedov(4, 16, 8, L=0.5, sigma=0.01)[:2],
               "config0 K8": lambda: W.config0(0, 8, 8)[:2],
               "sedov K4": lambda: W.sedov(1, 9, 4, L=0.4, sigma=0.02)[:2],
               "3-D blast K8": blast_3d_k8}[case]()
    p = W.Params()
    s = sedg.Solver(mesh, p)
    ug = _t(u)
    d = torch.zeros_like(ug)
    ab = torch.zeros(mesh.dof, dtype=torch.float64, device=DEV)
    dg = s.diagnose(ug, d, ab)
    s.check()
    s.close()
    d_o, info = O.rhs(mesh, p, u, full=True)
    assert rel_err(d.cpu().numpy(), d_o) <= RHS_TOL
    al, be = info["alpha"], info["beta"]
    assert dg["fallbacks"] == info["fallbacks"]
    assert dg["squeezed"] == int((be < 1.0).sum()) and dg["beta_rejected"] == int((be < p.beta_L).sum())
    ab_o = O.alpha_bar(mesh, p, al)
    assert np.abs(ab.cpu().numpy().reshape(ab_o.shape) - ab_o).max() <= 1e-13
    assert abs(dg["alpha_bar_mean"] - ab_o.mean()) <= 1e-12 and abs(dg["alpha_bar_min"] - ab_o.min()) <= 1e-13
    # lowest order carrying weight, per element, from the oracle's factors
    K, dim = mesh.K, mesh.dim
    levels, n = [], K
    while n >= 2:
        levels.append(n)
        n //= 2
    hist = {"FV": 0, "O2": 0, "O4": 0, "O8": 0}
    for e in range(mesh.nel):
        low = None
        for cell in np.ndindex(*([K] * dim)):     # (.., j, i): i along x
            prod, off = 1.0, 0
            for n in levels:
                ns = K // n
                q = sum((cell[dim - 1 - a] // n) * ns ** a for a in range(dim))
                a = al[e, off + q]
                if a * prod != 0.0:
                    low = n if low is None or n < low else low
                prod *= 1.0 - a
                off += ns ** dim
            if prod != 0.0:
                low = 1
        hist["FV" if low == 1 else "O%d" % low] += 1
    say("  diagnose %s: %s, fallbacks %d, squeezed %d, rejected %d, abar mean %.3f"
        % (case, dg["elems_by_lowest_order"], dg["fallbacks"], dg["squeezed"], dg["beta_rejected"], dg["alpha_bar_mean"]))
    assert dg["elems_by_lowest_order"] == hist
    assert dg["fallbacks"] > 0 or case != "sedov narrow"


def test_rk_step_frozen_matches_oracle_frozen_steps():
    """Two steps of the frozen map in the library against the same steps composed from
    the oracle's frozen right-hand side (factors and squeezing parameters of each stage
    from the adaptive run's tape)."""
    mesh, u, _ = W.sedov(2, 8, 8, L=0.3, sigma=0.03)
    p = W.Params()
    s = sedg.Solver(mesh, p)
    u0 = _t(u).reshape(-1)
    dts = torch.zeros(2, dtype=torch.float64, device=DEV)
    uT = u0.clone()
    s.rk_step(uT, 2, 0.0, dts)
    s.check()
    frozen = ADJ.record_frozen(s, u0, dts)
    # a perturbed state, so that the frozen factors are not the state's own
    up = u0 * (1.0 + 1e-7 * torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, u0.numel())).to(DEV))
    got = ADJ.frozen_evolve(s, up, frozen, dts).cpu().numpy().reshape(u.shape)
    assert torch.allclose(ADJ.frozen_evolve(s, u0, frozen, dts), uT, rtol=0, atol=1e-12 * float(uT.abs().max()))
    s.check()
    s.close()
    x = up.cpu().numpy().reshape(u.shape)
    fz = frozen.cpu().numpy()
    A = fz.shape[2]
    for j, dt in enumerate(dts.cpu().numpy()):
        al = [fz[j, k].reshape(mesh.nel, A // mesh.nel) for k in range(3)]
        be = [fz[j, 3 + k].reshape(mesh.nel, A // mesh.nel) for k in range(3)]
        L = O.rhs_frozen(mesh, p, x, al[0], be[0])
        x1 = x + dt * L
        L = O.rhs_frozen(mesh, p, x1, al[1], be[1])
        x2 = 0.75 * x + 0.25 * (x1 + dt * L)
        L = O.rhs_frozen(mesh, p, x2, al[2], be[2])
        x = (1.0 / 3.0) * x + (2.0 / 3.0) * (x2 + dt * L)
    err = rel_err(got, x)
    say("  frozen steps vs oracle rel_err=%.3e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("K", [4, 8])
def test_rk54_steps_match_oracle(K):
    """SSP-RK(5,4), the paper's integrator: 100 steps at CFL 0.8 within 1e-9 of the
    oracle's, step sizes (functions of the state) within 1e-11 (K = 4: the config-0 jump
    on 16x16 elements; K = 8: the narrow blast of 16x16 elements, as the config-0 jump at
    K = 8 is no multi-step case); in RANDOM mode the five stages of every step log the
    oracle's draws."""
    mesh, u, _ = W.config0(0, 16, 4) if K == 4 else W.sedov(4, 16, 8, L=0.5, sigma=0.01)
    p = W.Params(cfl=0.8, integrator=sedg.SEDG_SSPRK54)
    u_o, dts_o = O.rk3(mesh, p, u, 100)
    s = sedg.Solver(mesh, p)
    ug = _t(u)
    dts = torch.zeros(100, dtype=torch.float64, device=DEV)
    s.rk_step(ug, 100, 0.0, dts)
    s.check()
    err = rel_err(ug.cpu().numpy(), u_o)
    dterr = np.abs(dts.cpu().numpy() - dts_o).max() / dts_o.max()
    say("  ssp-rk(5,4) K=%d 100 steps rel_err=%.3e dt_err=%.3e" % (K, err, dterr))
    assert err <= STATE_TOL and dterr <= 1e-11
    # the step tape and the adjoint steps are SSP-RK3 only
    tape = torch.empty(s.tape_len, dtype=torch.float64, device=DEV)
    with pytest.raises(sedg.SedgError) as ei:
        s.rk_step_tape(ug, dts[:1], tape)
    assert ei.value.code == sedg.SEDG_EUNSUPPORTED
    s.close()
    pr = W.Params(cfl=0.8, integrator=sedg.SEDG_SSPRK54, mode=W.RANDOM, seed=3)
    mesh, u, _ = W.config0(0, 8, K)
    u_o, _ = O.rk3(mesh, pr, u, 10)
    s = sedg.Solver(mesh, pr)
    A = s.alpha_len
    ug = _t(u)
    alog = torch.zeros(50 * A, dtype=torch.float64, device=DEV)
    s.rk_step(ug, 10, 0.0, None, alog)
    s.check()
    assert rel_err(ug.cpu().numpy(), u_o) <= STATE_TOL
    la = alog.view(50, mesh.nel, A // mesh.nel).cpu().numpy()
    for d in (0, 4, 5, 49):
        assert np.array_equal(la[d], random_factors(pr.seed, d, mesh.nel, A // mesh.nel)), d
    s.close()


RC_CASES = [(2, 4, [5, 3], 0), (2, 8, [4, 3], 0), (2, 8, [3, 2], 1), (3, 4, [3, 2, 2], 0), (3, 8, [2, 2, 1], 0)]


@pytest.mark.parametrize("dim,K,ne,fam", RC_CASES)
def test_refine_coarsen_match_oracle(dim, K, ne, fam):
    """Blended refinement and coarsening (App., eq. 3D-refinement, 3D-coarsening) with
    random factors on every level against the oracle's, within 1e-13 of the state's
    magnitude; totals conserved."""
    mesh = W.Mesh(dim, K, ne, [0.0] * dim, [1.0] * dim, [0] * dim, family=fam)
    p = W.Params()
    rng = np.random.default_rng(11)
    u = np.zeros(mesh.shape())
    u[0] = 1.0 + 0.5 * rng.uniform(size=u[0].shape)
    for a in range(dim):
        u[1 + a] = 0.2 * rng.standard_normal(u[0].shape)
    u[dim + 1] = 3.0 + rng.uniform(size=u[0].shape)
    A = W.alpha_len(mesh, p)
    fm = O.fine_mesh(mesh)
    al = rng.uniform(size=(mesh.nel, A))
    alf = rng.uniform(size=(fm.nel, A))
    s = sedg.Solver(mesh, p)
    uf = torch.zeros(fm.nvar * fm.dof, dtype=torch.float64, device=DEV)
    s.refine(_t(u), _t(al), uf)
    uc = torch.zeros(s.state_len, dtype=torch.float64, device=DEV)
    s.coarsen(uf, _t(alf), uc)
    s.check()
    s.close()
    uf_o = O.refine(mesh, p, u, al)
    uc_o = O.coarsen(mesh, p, uf_o, alf)
    ef = np.abs(uf.cpu().numpy().reshape(uf_o.shape) - uf_o).max() / np.abs(uf_o).max()
    ec = np.abs(uc.cpu().numpy().reshape(uc_o.shape) - uc_o).max() / np.abs(uc_o).max()
    say("  refine/coarsen %dD K=%d fam %d: refine rel %.2e, coarsen rel %.2e" % (dim, K, fam, ef, ec))
    assert ef <= 1e-13 and ec <= 1e-13
    tot = u.reshape(mesh.nvar, -1).sum(1)
    assert np.allclose(uf.view(fm.nvar, -1).sum(1).cpu().numpy() / 2 ** dim, tot, rtol=1e-13, atol=0)
