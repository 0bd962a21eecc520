"""GPU parity of the frozen right-hand side and its adjoint (vector-Jacobian
product) against the oracle, of the transposed SSP-RK3 step against the oracle's
adjoint composed over the three stages, and of the checkpointed
torch.autograd evolution against central differences of the frozen forward map.

The blending factors and squeezing parameters fed to both sides come from the
oracle (or from a seeded generator); the adjoint states are seeded normals."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_03338_amd import sedg, workloads as W
from tests.parity import DEV, blast_3d_k8, check_factors, say

pytestmark = pytest.mark.gpu

# one frozen right-hand side / one adjoint: the joint relative norm of tests/parity.py
FROZEN_TOL = 1e-12
ADJ_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sedg.load()
    yield


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _rel(g, o):
    return np.abs(np.asarray(g) - np.asarray(o)).max() / np.abs(np.asarray(o)).max()


def _oracle_frozen_inputs(mesh, u, kind, seed=0):
    """(alpha, beta): the oracle's own at u, or seeded factors with the oracle's beta."""
    _, info = O.rhs(mesh, W.Params(), u, full=True)
    al, be = info["alpha"], info["beta"]
    rng = np.random.default_rng(seed)
    if kind == "random":
        al = rng.uniform(0.0, 1.0, al.shape)
    elif kind == "mid":
        al = rng.uniform(0.2, 0.8, al.shape)
    elif kind == "fv":
        al = np.zeros_like(al)
    return al, be


def _cases():
    out = []
    m, u, _ = W.config0(0, 16, 4)
    out.append(("config0 K4 adaptive", m, u, "adaptive"))
    m, u, _ = W.config0(1, 6, 8)
    out.append(("config0 K8 random", m, u, "random"))
    out.append(("config0 K8 adaptive", m, u, "adaptive"))
    m, u, _ = W.sedov(2, 6, 8, L=0.3, sigma=0.03)
    out.append(("sedov resolved adaptive", m, u, "adaptive"))
    out.append(("sedov resolved mid", m, u, "mid"))
    out.append(("sedov resolved fv", m, u, "fv"))
    m, u, _ = W.sedov(1, 7, 4, L=0.3, sigma=0.03)
    out.append(("sedov K4 7x7 mid", m, u, "mid"))
    m, u, _ = W.pressure_pulse(0, 6, 8)
    out.append(("pulse K8 adaptive", m, u, "adaptive"))
    return out


def _cases_3d():
    """3-D cases of the frozen map (the 3-D K = 8 adjoint is not built): the per-level
    sub-element means of a z layer's level-4 and level-2 sub-elements cross the
    element's wavefronts at K = 8."""
    out = []
    m, u, _ = W.shear_layer_3d(0, 2, 8)
    out.append(("3-D shear K8 adaptive", m, np.ascontiguousarray(u.numpy()), "adaptive"))
    out.append(("3-D shear K8 random", m, np.ascontiguousarray(u.numpy()), "random"))
    m, u = blast_3d_k8()
    out.append(("3-D blast K8 mid", m, u, "mid"))
    m, u, _ = W.shear_layer_3d(1, 3, 4)
    out.append(("3-D shear K4 mid", m, np.ascontiguousarray(u.numpy()), "mid"))
    return out


CASES = _cases()
FROZEN_CASES = CASES + _cases_3d()


@pytest.mark.parametrize("case", range(len(FROZEN_CASES)), ids=[c[0] for c in FROZEN_CASES])
def test_frozen_rhs_matches_oracle(case):
    label, mesh, u, kind = FROZEN_CASES[case]
    al, be = _oracle_frozen_inputs(mesh, u, kind)
    d_o = O.rhs_frozen(mesh, W.Params(), u, al, be)
    s = sedg.Solver(mesh, W.Params())
    dg = torch.zeros_like(_t(u))
    s.rhs_frozen(_t(u), _t(al), _t(be), dg)
    s.check()
    err = _rel(dg.cpu().numpy(), d_o)
    say("  frozen %-26s rel_err=%.3e" % (label, err))
    assert err <= FROZEN_TOL
    s.close()


@pytest.mark.parametrize("K,ne", [(4, 16), (8, 8)])
def test_frozen_rhs_equals_adaptive(K, ne):
    """With the factors the adaptive evaluation chose, the frozen map reproduces it
    up to rounding: the residual kernel is the same, but the element-face states
    and means come from the preparation kernel instead of the analyse kernel, where
    the compiler may fuse multiply-adds differently."""
    mesh, u, _ = W.sedov(0, ne, K, L=0.3, sigma=0.03)
    s = sedg.Solver(mesh, W.Params())
    ug = _t(u)
    d1 = torch.zeros_like(ug)
    al = torch.zeros(s.alpha_len, dtype=torch.float64, device=DEV)
    be = torch.zeros_like(al)
    s.rhs(ug, d1, al, be)
    d2 = torch.zeros_like(ug)
    s.rhs_frozen(ug, al, be, d2)
    s.check()
    err = float((d1 - d2).abs().max() / d1.abs().max())
    say("  frozen vs adaptive K%d: rel %.2e" % (K, err))
    assert err <= 1e-13
    s.close()


def _gpu_adjoint(mesh, u, al, be, lam):
    s = sedg.Solver(mesh, W.Params())
    out = torch.zeros_like(_t(u))
    s.adjoint_rhs(_t(u), _t(al), _t(be), _t(lam), out)
    s.check()
    r = out.cpu().numpy()
    s.close()
    return r


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_adjoint_rhs_matches_oracle(case):
    label, mesh, u, kind = CASES[case]
    al, be = _oracle_frozen_inputs(mesh, u, kind)
    lam = np.random.default_rng(11).standard_normal(u.shape)
    a_o = O.adjoint_rhs(mesh, W.Params(), u, al, be, lam)
    a_g = _gpu_adjoint(mesh, u, al, be, lam)
    err = _rel(a_g, a_o)
    say("  adjoint %-25s rel_err=%.3e" % (label, err))
    assert err <= ADJ_TOL


def test_adjoint_single_periodic_element():
    """One periodic element: both element faces are the element's own seam."""
    K = 8
    mesh = W.Mesh(2, K, [1, 1], [0, 0], [1, 1], [0, 0])
    u = W.density_wave(mesh, vel=(0.3, -0.2, 0), amp=0.2)
    al, be = _oracle_frozen_inputs(mesh, u, "random", seed=4)
    lam = np.random.default_rng(12).standard_normal(u.shape)
    err = _rel(_gpu_adjoint(mesh, u, al, be, lam), O.adjoint_rhs(mesh, W.Params(), u, al, be, lam))
    say("  adjoint single element rel_err=%.3e" % err)
    assert err <= ADJ_TOL


def test_adjoint_3d_k4():
    mesh = W.Mesh(3, 4, [3, 2, 2], [0.0] * 3, [1.0] * 3, [0, 1, 0])
    rng = np.random.default_rng(3)
    u = np.zeros(mesh.shape())
    u[0] = 1.0 + 0.5 * rng.uniform(size=u[0].shape)
    u[1] = 0.3 * u[0]
    u[2] = -0.2 * u[0]
    u[4] = (1.0 + 0.5 * rng.uniform(size=u[0].shape)) / 0.4 + 0.5 * 0.13 * u[0]
    al, be = _oracle_frozen_inputs(mesh, u, "random", seed=5)
    lam = rng.standard_normal(u.shape)
    err = _rel(_gpu_adjoint(mesh, u, al, be, lam), O.adjoint_rhs(mesh, W.Params(), u, al, be, lam))
    say("  adjoint 3-D K4 rel_err=%.3e" % err)
    assert err <= ADJ_TOL


# (label, K, parameters, sub-cell family, workload)
PARAM_VARIANTS = [("K8 top level 4", 8, dict(top_level=4), W.GAUSS, "sedov"),
                  ("K8 levels 8+2", 8, dict(level_mask=(1 << 3) | (1 << 1)), W.GAUSS, "sedov"),
                  ("K8 single level 4", 8, dict(level_mask=1 << 2), W.GAUSS, "sedov"),
                  ("K8 LGL", 8, {}, W.LGL, "config0"), ("K8 LGL level 4", 8, dict(level_mask=1 << 2), W.LGL, "config0"),
                  ("K4 LGL top level 2", 4, dict(top_level=2), W.LGL, "config0")]


def _param_variant_state(K, family, workload):
    """Resolved blast (squeezed sub-elements) for Gauss sub-cells.  LGL sub-cells put
    nodes on element faces, where the blast's squeeze binds at zero pressure and the
    config-0 jump samples a pure contact (equal velocity and sound speed on both
    sides): the frozen map has kinks there (the sound speed's square root at zero, the
    Einfeldt minimum of two equal estimates with different states), so LGL uses the
    config-0 state with seeded 1e-3 relative noise on every cell mean, which moves
    every face state off those sets."""
    import dataclasses
    if workload == "sedov":
        mesh, u, _ = W.sedov(3, 6, K, L=0.3, sigma=0.03)
    else:
        mesh, u, _ = W.config0(1, 6, K)
        u = u * (1.0 + 1e-3 * np.random.default_rng(7).standard_normal(u.shape))
    return dataclasses.replace(mesh, family=family), u


@pytest.mark.parametrize("variant", range(len(PARAM_VARIANTS)), ids=[v[0] for v in PARAM_VARIANTS])
def test_frozen_and_adjoint_param_variants(variant):
    """Reduced level hierarchies (a lower top level, level masks) and LGL sub-cells:
    the frozen map and its adjoint against the oracle, with the oracle's own factors,
    with seeded ones and with pure DG (alpha = 1)."""
    label, K, kw, family, workload = PARAM_VARIANTS[variant]
    prm = W.Params(**kw)
    mesh, u = _param_variant_state(K, family, workload)
    _, info = O.rhs(mesh, prm, u, full=True)
    rng = np.random.default_rng(31 + variant)
    lam = rng.standard_normal(u.shape)
    for kind in ("adaptive", "random", "dg"):
        al = {"adaptive": info["alpha"], "random": rng.uniform(0.0, 1.0, info["alpha"].shape),
              "dg": np.ones_like(info["alpha"])}[kind]
        be = info["beta"]
        s = sedg.Solver(mesh, prm)
        assert s.alpha_len == al.size
        dg = torch.zeros_like(_t(u))
        s.rhs_frozen(_t(u), _t(al), _t(be), dg)
        lg = torch.zeros_like(_t(u))
        s.adjoint_rhs(_t(u), _t(al), _t(be), _t(lam), lg)
        s.check()
        s.close()
        ef = _rel(dg.cpu().numpy(), O.rhs_frozen(mesh, prm, u, al, be))
        ea = _rel(lg.cpu().numpy(), O.adjoint_rhs(mesh, prm, u, al, be, lam))
        say("  %-20s %-8s frozen %.2e adjoint %.2e" % (label, kind, ef, ea))
        assert ef <= FROZEN_TOL and ea <= ADJ_TOL


def test_adjoint_unsupported_and_invalid():
    mesh = W.Mesh(3, 8, [1, 1, 1], [0.0] * 3, [1.0] * 3, [0, 0, 0])
    s = sedg.Solver(mesh, W.Params())
    x = torch.ones(s.state_len, dtype=torch.float64, device=DEV)
    a = torch.ones(s.alpha_len, dtype=torch.float64, device=DEV)
    with pytest.raises(sedg.SedgError) as ei:
        s.adjoint_rhs(x, a, a, x.clone(), torch.zeros_like(x))
    assert ei.value.code == sedg.SEDG_EUNSUPPORTED
    s.close()
    mesh, u, _ = W.config0(0, 4, 4)
    s = sedg.Solver(mesh, W.Params())
    x = _t(u).reshape(-1)
    a = torch.ones(s.alpha_len, dtype=torch.float64, device=DEV)
    with pytest.raises(sedg.SedgError) as ei:
        s.adjoint_rhs(x, a, a, x, x)          # output aliases the input
    assert ei.value.code == sedg.SEDG_EINVAL
    s.close()


# ---------------------------------------------------------------------------
# transposed RK3 step
# ---------------------------------------------------------------------------

def _oracle_step_adjoint(mesh, u0, dt, lam3):
    """The oracle's stage states (adaptive factors at each stage) and the transposed
    step composed from the oracle's adjoint right-hand side."""
    p = W.Params()
    L0, i0 = O.rhs(mesh, p, u0, full=True)
    u1 = u0 + dt * L0
    L1, i1 = O.rhs(mesh, p, u1, full=True)
    u2 = 0.75 * u0 + 0.25 * (u1 + dt * L1)
    _, i2 = O.rhs(mesh, p, u2, full=True)
    A = lambda u, info, lam: O.adjoint_rhs(mesh, p, u, info["alpha"], info["beta"], lam)
    l2 = (2.0 / 3.0) * (lam3 + dt * A(u2, i2, lam3))
    l1 = 0.25 * (l2 + dt * A(u1, i1, l2))
    return (1.0 / 3.0) * lam3 + 0.75 * l2 + l1 + dt * A(u0, i0, l1)


@pytest.mark.parametrize("name", ["config0", "sedov", "sedov K4", "pulse"])
def test_adjoint_rk_step_matches_oracle(name):
    """The blasts here keep every stage state permissible at the CFL step (squeezed
    sub-elements in both)."""
    if name == "config0":
        mesh, u0, _ = W.config0(2, 8, 4)
    elif name == "sedov":
        mesh, u0, _ = W.sedov(1, 8, 8)
    elif name == "sedov K4":
        mesh, u0, _ = W.sedov(2, 8, 4, L=0.5, sigma=0.05)
    else:
        mesh, u0, _ = W.pressure_pulse(1, 6, 8)
    dt = O.max_dt(mesh, W.Params(), u0)
    lam3 = np.random.default_rng(21).standard_normal(u0.shape)
    ref = _oracle_step_adjoint(mesh, u0, dt, lam3)
    s = sedg.Solver(mesh, W.Params())
    ug = _t(u0).reshape(-1)
    tape = torch.zeros(s.tape_len, dtype=torch.float64, device=DEV)
    dtd = torch.tensor([dt], dtype=torch.float64, device=DEV)
    s.rk_step_tape(ug, dtd, tape)
    lam = _t(lam3).reshape(-1)
    s.adjoint_rk_step(tape, dtd, lam)
    s.check()
    err = _rel(lam.cpu().numpy().reshape(u0.shape), ref)
    say("  adjoint RK step %-10s rel_err=%.3e" % (name, err))
    assert err <= ADJ_TOL
    s.close()


def test_tape_step_reproduces_rk_step():
    """Taped steps with the logged step sizes reproduce sedg_rk_step bit for bit."""
    mesh, u0, _ = W.sedov(0, 8, 8, L=0.3, sigma=0.03)
    s = sedg.Solver(mesh, W.Params())
    ua = _t(u0).reshape(-1)
    ub = ua.clone()
    log = torch.zeros(3, dtype=torch.float64, device=DEV)
    s.rk_step(ua, 3, 0.0, log)
    tapes = torch.zeros((3, s.tape_len), dtype=torch.float64, device=DEV)
    s.rk_step_tape(ub, log, tapes)
    s.check()
    assert torch.equal(ua, ub)
    # the last tape's initial state is the state after two steps
    uc = _t(u0).reshape(-1)
    s.rk_step(uc, 2, 0.0, None)
    s.check()
    assert torch.equal(tapes[2, :uc.numel()], uc)
    s.close()


# ---------------------------------------------------------------------------
# checkpointed autograd evolution vs central differences of the frozen map
# ---------------------------------------------------------------------------

def test_autograd_evolution_finite_differences():
    """Pulse workload (periodic, K = 8) on 8x8 elements, 25 steps with a checkpoint
    every 7 steps (ragged last segment).  J = sum of rho^2 |cell| over the centre
    window [0.4, 0.6]^2; directional derivatives along 8 seeded unit directions
    against central differences of the frozen map at eps = 1e-6 (relative to the
    state's magnitude)."""
    from paper_2011_03338_amd import adjoint as ADJ
    mesh, u0n, _ = W.pressure_pulse(0, 8, 8)
    s = sedg.Solver(mesh, W.Params())
    u0 = _t(u0n).reshape(-1)
    G = mesh.grid
    xc = (np.arange(G[0]) + 0.5) / G[0]
    yc = (np.arange(G[1]) + 0.5) / G[1]
    win = _t(((yc[:, None] >= 0.4) & (yc[:, None] <= 0.6) & (xc[None, :] >= 0.4) & (xc[None, :] <= 0.6)).astype(float))
    cell = 1.0 / (G[0] * G[1])

    def J(u):
        return (u[:G[0] * G[1]].reshape(G[1], G[0]) ** 2 * win).sum() * cell

    nsteps, every = 25, 7
    x = u0.clone().requires_grad_(True)
    uT = ADJ.evolve(x, s, nsteps, every)
    J(uT).backward()
    grad = x.grad.detach()
    dts = ADJ.dt_log_of(uT)[:nsteps].clone()
    frozen = ADJ.record_frozen(s, u0, dts)
    assert torch.allclose(ADJ.frozen_evolve(s, u0, frozen, dts), uT.detach(), rtol=0, atol=1e-12)
    rng = np.random.default_rng(17)
    scale = u0.abs()
    errs = []
    for k in range(8):
        v = _t(rng.standard_normal(u0.shape[0])) * scale
        v = v / v.norm()
        eps = 1e-6 * u0.norm()
        jp = J(ADJ.frozen_evolve(s, u0 + eps * v, frozen, dts))
        jm = J(ADJ.frozen_evolve(s, u0 - eps * v, frozen, dts))
        fd = float((jp - jm) / (2 * eps))
        ad = float((grad * v).sum())
        errs.append(abs(fd - ad) / abs(ad))
    say("  autograd FD rel errors: " + " ".join("%.1e" % e for e in errs))
    # central differences at this step carry ~1e-7..1e-6 of truncation and rounding
    assert max(errs) <= 2e-6
    s.close()


def test_full_size_adjoint_windows():
    """The adjoint workload's size and state (128x128 periodic elements, K = 8, pressure
    pulse): the adjoint right-hand side at the adaptive factors, with a seeded adjoint
    state, against the oracle's on 5x5-element windows (outflow edges on the cut); the
    interior 3x3 elements only see fluxes between window elements.  The oracle's adjoint
    runs on the factors and squeezing parameters of its own forward analysis of the
    window (element-local, so the cut does not change them), checked against the GPU's
    factors first; an element whose decision lies at a threshold gets the oracle's
    factors on the GPU side too."""
    mesh, u, _ = W.pressure_pulse(0, 128, 8)
    p = W.Params()
    s = sedg.Solver(mesh, p)
    ug = _t(u)
    d = torch.zeros_like(ug)
    al = torch.zeros(s.alpha_len, dtype=torch.float64, device=DEV)
    be = torch.zeros_like(al)
    s.rhs(ug, d, al, be)
    lam = np.random.default_rng(41).standard_normal(u.shape)
    out = torch.zeros_like(ug)
    s.adjoint_rhs(ug, al, be, _t(lam), out)
    s.check()
    s.close()
    A = W.alpha_len(mesh, p)
    aln = al.cpu().numpy().reshape(128, 128, A)
    ben = be.cpu().numpy().reshape(128, 128, A)
    g = out.cpu().numpy()
    K, h = 8, 1.0 / 128
    rng = np.random.default_rng(3)
    centres = [(72, 49), (64, 64), (56, 40)] + [tuple(int(x) for x in rng.integers(2, 126, 2)) for _ in range(3)]
    for (ex, ey) in centres:
        x0, y0 = ex - 2, ey - 2
        wm = W.Mesh(2, K, [5, 5], [x0 * h, y0 * h], [(x0 + 5) * h, (y0 + 5) * h], [1, 1])
        sl = (slice(None), slice(None), slice(y0 * K, (y0 + 5) * K), slice(x0 * K, (x0 + 5) * K))
        uw = np.ascontiguousarray(u[sl])
        _, info = O.rhs(wm, p, uw, full=True)
        gal = np.ascontiguousarray(aln[y0:y0 + 5, x0:x0 + 5].reshape(25, A))
        gbe = np.ascontiguousarray(ben[y0:y0 + 5, x0:x0 + 5].reshape(25, A))
        exempt = check_factors(gal, gbe, info, p, "adjoint window (%d,%d)" % (ex, ey))
        o = O.adjoint_rhs(wm, p, uw, info["alpha"], info["beta"], np.ascontiguousarray(lam[sl]))
        oi = o[:, :, K:4 * K, K:4 * K]
        gw = g
        if exempt:
            # the oracle's decisions at the threshold elements, fed to the GPU's adjoint
            a2, b2 = aln.copy(), ben.copy()
            a2[y0:y0 + 5, x0:x0 + 5] = info["alpha"].reshape(5, 5, A)
            b2[y0:y0 + 5, x0:x0 + 5] = info["beta"].reshape(5, 5, A)
            s2 = sedg.Solver(mesh, p)
            o2 = torch.zeros_like(ug)
            s2.adjoint_rhs(ug, _t(a2.reshape(-1)), _t(b2.reshape(-1)), _t(lam), o2)
            s2.check()
            s2.close()
            gw = o2.cpu().numpy()
        gi = gw[:, :, (y0 + 1) * K:(y0 + 4) * K, (x0 + 1) * K:(x0 + 4) * K]
        err = np.abs(gi - oi).max() / np.abs(oi).max()
        say("  adjoint window (%d,%d) rel_err=%.3e exempt=%d" % (ex, ey, err, len(exempt)))
        assert err <= ADJ_TOL
