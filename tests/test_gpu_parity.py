"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the
same seeded inputs.  Run on an MI355X with  pytest -m gpu."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_03338_amd import sedg, workloads as W
from tests.parity import (DEV, RHS_TOL, STATE_TOL, blast_3d_k8, check_factors, compare_rhs, factor_noise, gpu_rhs,
                          rel_err, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sedg.load()
    yield


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rhs_config0(seed):
    """2-D periodic 16x16 elements, K = 4, density wave with a seeded jump."""
    mesh, u, _ = W.config0(seed, 16, 4)
    compare_rhs(mesh, W.Params(), u, "config0 seed%d" % seed)


@pytest.mark.parametrize("seed", [0, 3])
def test_rhs_config0_k8(seed):
    mesh, u, _ = W.config0(seed, 8, 8)
    compare_rhs(mesh, W.Params(), u, "config0 K8 seed%d" % seed)


@pytest.mark.parametrize("K,ne", [(8, 8), (8, 13), (4, 16), (4, 7)])
def test_rhs_sedov(K, ne):
    """Sedov-type blast with outflow boundaries; odd element counts leave a ragged
    last workgroup."""
    mesh, u, _ = W.sedov(1, ne, K)
    compare_rhs(mesh, W.Params(), u, "sedov K%d ne%d" % (K, ne))


def test_rhs_sedov_resolved():
    """The blast resolved over a few elements (mixed levels, squeezes, fallbacks)."""
    mesh, u, _ = W.sedov(2, 12, 8, L=0.3, sigma=0.03)
    compare_rhs(mesh, W.Params(), u, "sedov resolved")


@pytest.mark.parametrize("K,ne,bc", [(8, [1, 3], [0, 1]), (4, [1, 1], [0, 0]), (8, [2, 1], [1, 0])])
def test_rhs_single_element_periodic_axis(K, ne, bc):
    """One periodic element along an axis: its low and high element faces are the same
    face, whose common flux is computed once and read by both sides."""
    mesh = W.Mesh(2, K, ne, [0, 0], [0.3 * ne[0], 0.3 * ne[1]], bc)
    rng = np.random.default_rng(21 + K)
    u = np.zeros(mesh.shape())
    g = mesh.grid
    u[0] = 1.0 + 0.5 * rng.uniform(size=(1, g[1], g[0]))
    u[1] = 0.3 * u[0]
    u[2] = 0.1 * u[0]
    u[3] = (1.0 + 0.5 * rng.uniform(size=(1, g[1], g[0]))) / 0.4 + 0.5 * 0.1 * u[0]
    compare_rhs(mesh, W.Params(), u, "single periodic element K=%d %s" % (K, ne))


def test_rhs_nonsquare_ragged():
    mesh, u0, _ = W.config0(4, 6, 8)
    mesh = W.Mesh(2, 8, [5, 3], [0, 0], [1.0, 0.6], [0, 1])
    rng = np.random.default_rng(9)
    u = np.zeros(mesh.shape())
    g = mesh.grid
    u[0] = 1.0 + 0.5 * rng.uniform(size=(1, g[1], g[0]))
    u[1] = 0.2 * u[0]
    u[2] = -0.1 * u[0]
    u[3] = (1.0 + 0.5 * rng.uniform(size=(1, g[1], g[0]))) / 0.4 + 0.5 * 0.05 * u[0]
    compare_rhs(mesh, W.Params(), u, "5x3 random")


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("mode", [W.FORCE_DG, W.FORCE_FV, W.EXTERNAL])
def test_rhs_modes(K, mode):
    mesh, u, _ = W.config0(5, 6 if K == 8 else 10, K)
    p = W.Params(mode=mode)
    if mode == W.EXTERNAL:
        rng = np.random.default_rng(17)
        A = W.alpha_len(mesh, p)
        al = rng.uniform(0, 1, size=(mesh.nel, A))
        d_o = O.rhs(mesh, p, u, alpha_in=al)
        d_g, a_g, _ = gpu_rhs(mesh, p, u, al)
        assert np.array_equal(a_g, al)
        err = rel_err(d_g, d_o)
        say("  parity external K%d rel_err=%.3e" % (K, err))
        assert err <= RHS_TOL
    else:
        compare_rhs(mesh, p, u, "mode%d K%d" % (mode, K))


def test_rhs_lgl_nodes():
    mesh, u, _ = W.config0(6, 6, 8)
    mesh.family = W.LGL
    compare_rhs(mesh, W.Params(), u, "LGL K8")


@pytest.mark.parametrize("top", [4, 2])
def test_rhs_dgfv_top_level(top):
    mesh, u, _ = W.sedov(3, 8, 8, L=0.5, sigma=0.05)
    compare_rhs(mesh, W.Params(top_level=top), u, "DGFV%d" % top)


def test_rhs_indicator_floor_variant():
    """The indicator's denominator floor below the data's scale (a variant, not the
    paper's 1): a narrow blast at K = 8 and K = 4."""
    for K in (8, 4):
        mesh, u, _ = W.sedov(4, 12, K, L=0.5, sigma=0.01)
        compare_rhs(mesh, W.Params(sigma_floor=1e-14), u, "floor 1e-14 K=%d" % K)


def test_rhs_single_level_mask():
    mesh, u, _ = W.sedov(3, 8, 8, L=0.5, sigma=0.05)
    compare_rhs(mesh, W.Params(level_mask=1 << 3), u, "single level")


@pytest.mark.parametrize("K,ne", [(4, 3), (8, 2)])
def test_rhs_3d(K, ne):
    mesh, u, _ = W.shear_layer_3d(0, ne, K)
    u = u.numpy()
    compare_rhs(mesh, W.Params(), u, "3d KH K%d" % K)
    p = W.Params(mode=W.EXTERNAL)
    rng = np.random.default_rng(23)
    al = rng.uniform(0, 1, size=(mesh.nel, W.alpha_len(mesh, p)))
    err = rel_err(gpu_rhs(mesh, p, u, al)[0], O.rhs(mesh, p, u, alpha_in=al))
    say("  parity 3d external K%d rel_err=%.3e" % (K, err))
    assert err <= RHS_TOL


def test_rhs_3d_outflow_jump():
    mesh = W.Mesh(3, 4, [3, 2, 2], [0, 0, 0], [1, 1, 1], [1, 0, 1])
    g = mesh.grid
    x = (np.arange(g[0]) + 0.5) / g[0]
    u = np.zeros(mesh.shape())
    u[0] = np.where(x < 0.45, 1.0, 0.2)[None, None, :]
    u[1] = 0.3 * u[0]
    u[4] = np.where(x < 0.45, 2.0, 0.3)[None, None, :] / 0.4 + 0.5 * 0.09 * u[0]
    compare_rhs(mesh, W.Params(), u, "3d outflow jump")


def test_rhs_3d_k8_blast_squeezed():
    """A concentrated 3-D blast (4^3 K = 8 elements over [-1/2, 1/2]^3, outflow, Gaussian
    energy of width 0.04 over p0 = 1e-5): squeezed sub-elements on every level (8 on the
    top level, 24 on level 4, 129 on level 2 in the oracle), blended factors and
    interface-safety fallbacks; one right-hand side, factors and squeezing parameters
    against the oracle's (the per-level sub-element means and minima of a z layer's
    level-4 and level-2 sub-elements cross the element's wavefronts)."""
    mesh, u = blast_3d_k8()
    _, info = O.rhs(mesh, W.Params(), u, full=True)
    b = info["beta"]
    assert (b[:, 0] < 1).sum() > 0 and (b[:, 1:9] < 1).sum() > 0 and (b[:, 9:] < 1).sum() > 0
    compare_rhs(mesh, W.Params(), u, "3d K8 blast squeezed")


VARIANTS_3D = {
    "DGFV4": dict(top_level=4), "DGFV2": dict(top_level=2), "force_dg": dict(mode=W.FORCE_DG),
    "force_fv": dict(mode=W.FORCE_FV), "single_level": dict(level_mask=1 << 3),
    "random": dict(mode=W.RANDOM, seed=99), "floor_variant": dict(sigma_floor=1e-14),
}


# The floor variant is not run on the LGL blast: there the background's smoothness
# measures (about 1e-15) fall below the variant's floor of 1e-14, so a factor is 100 times
# a difference of rounding-size numbers divided by the floor; three evaluations in
# different arithmetic orders (the oracle, the GPU, numpy from the oracle's tables) give
# 0.661519, 0.661368 and 0.661459 for the same sub-element.  The paper's floor of 1
# rules this out; the variant is covered on the Gauss blast and the shear layer.
CASES_3D = [(st, v) for v in sorted(VARIANTS_3D) for st in ("blast", "shear", "blast_lgl")
            if not (st == "blast_lgl" and v == "floor_variant")]


@pytest.mark.parametrize("state,variant", CASES_3D)
def test_rhs_3d_k8_variants(state, variant):
    """The 3-D K = 8 kernels under every parameter that changes their control flow or
    tables (top levels 4 and 2, forced DG or FV, the single-level mask, random factors,
    the indicator floor variant) on the squeezed blast (Gauss and LGL nodes) and on the
    2^3-element shear layer: one right-hand side, factors and squeezing parameters
    against the oracle's (random factors: the same SplitMix64 draw on both sides).
    Some of these states are ill-conditioned in FP64: forced DG on the under-resolved
    shear layer squeezes whole elements to beta = 0, and the floor variant divides by
    smoothness measures of the background's rounding size, so that the oracle's own
    right-hand side (factors) moves by up to 1e-11 (1e-8) under a 1-ulp perturbation of
    its input.  As for the full-size windows, the bar is 1e-12 of the largest
    right-hand side, or 4 times that 1-ulp change where it is larger (both printed)."""
    if state == "shear":
        mesh, u, _ = W.shear_layer_3d(0, 2, 8)
        u = u.numpy()
    else:
        mesh, u = blast_3d_k8(W.LGL if state == "blast_lgl" else W.GAUSS)
    u = np.ascontiguousarray(u)
    p = W.Params(**VARIANTS_3D[variant])
    label = "3d K8 %s %s" % (state, variant)
    do, info = O.rhs(mesh, p, u, full=True)
    dg, ag, bg = gpu_rhs(mesh, p, u)
    exempt = check_factors(ag, bg, info, p, label, factor_noise(mesh, p, u, info))
    if exempt:
        # the oracle's decisions fed to both sides
        p = W.Params(**{**p.__dict__, "mode": W.EXTERNAL})
        do = O.rhs(mesh, p, u, alpha_in=info["alpha"])
        dg = gpu_rhs(mesh, p, u, info["alpha"])[0]
    sel = (slice(None),) * 4
    _window_compare(label + (" (%d exempt)" % len(exempt) if exempt else ""), dg, do,
                    _one_ulp_change(mesh, p, u, do, sel))


def test_rk3_100_steps_config0():
    """100 SSP-RK3 steps at CFL 0.5 on the 16x16, K = 4 case: state within 1e-9,
    step sizes within 1e-14."""
    mesh, u, _ = W.config0(0, 16, 4)
    p = W.Params(cfl=0.5)
    u_o, dts_o = O.rk3(mesh, p, u, 100)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u).to(DEV)
    dts = torch.zeros(100, dtype=torch.float64, device=DEV)
    s.rk_step(ug, 100, 0.0, dts)
    s.check()
    err = rel_err(ug.cpu().numpy(), u_o)
    dterr = np.abs(dts.cpu().numpy() - dts_o).max() / dts_o.max()
    say("  rk3 100 steps rel_err=%.3e dt_err=%.3e" % (err, dterr))
    assert err <= STATE_TOL and dterr <= 1e-14
    s.close()


def test_rk3_k8_blast_100_steps():
    """100 SSP-RK3 steps at CFL 0.5 of a K = 8 blast (16x16 elements over [-0.5, 0.5]^2)
    whose width (0.01) is under one element (0.0625): blended levels, squeezed
    sub-elements and interface-safety fallbacks at every step.  State within 1e-9 of
    the oracle's; step sizes, functions of the state, within 1e-11.  (The config-0 jump
    at K = 8 is no multi-step case: the oracle's own trajectory moves by 1e-8 within 48
    steps under a 1e-15 relative perturbation of its initial state, as indicator values
    cross thresholds.)"""
    case = "blast"
    mesh, u = W.sedov(4, 16, 8, L=0.5, sigma=0.01)[:2]
    p = W.Params(cfl=0.5)
    u_o, dts_o = O.rk3(mesh, p, u, 100)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u).to(DEV)
    dts = torch.zeros(100, dtype=torch.float64, device=DEV)
    s.rk_step(ug, 100, 0.0, dts)
    s.check()
    ugn = ug.cpu().numpy()
    err = rel_err(ugn, u_o)
    dterr = np.abs(dts.cpu().numpy() - dts_o).max() / dts_o.max()
    _, info = O.rhs(mesh, p, u_o, full=True)
    al = info["alpha"]
    say("  rk3 %s K8 16x16 100 steps rel_err=%.3e dt_err=%.3e; at step 100: %d of %d elements "
        "below pure top-level DG, %d squeezed sub-elements, %d fallbacks"
        % (case, err, dterr, int((al[:, 0] < 1.0).sum()), mesh.nel, int((info["beta"] < 1.0).sum()), info["fallbacks"]))
    assert (al[:, 0] < 1.0).sum() > 0
    assert err <= STATE_TOL and dterr <= 1e-11
    s.close()


def _jump_3d(K, ne):
    mesh = W.Mesh(3, K, ne, [0, 0, 0], [1, 1, 1], [W.OUTFLOW, W.PERIODIC, W.OUTFLOW])
    g = mesh.grid
    x = (np.arange(g[0]) + 0.5) / g[0]
    u = np.zeros(mesh.shape())
    u[0] = np.where(x < 0.45, 1.0, 0.2)[None, None, :]
    u[1] = 0.3 * u[0]
    u[4] = np.where(x < 0.45, 2.0, 0.3)[None, None, :] / 0.4 + 0.5 * 0.09 * u[0]
    return mesh, u


@pytest.mark.parametrize("case,steps", [("shear K4 4^3", 100), ("shear K8 2^3", 60), ("jump K8 4x2x2 outflow", 50),
                                        ("shear K8 2^3 SSP-RK(5,4)", 40)])
def test_rk3_3d_multistep(case, steps):
    """Whole SSP-RK3 steps in 3-D against the oracle: the shear layer on 4^3 K = 4 and
    2^3 K = 8 elements (at the end every K = 8 element is blended below pure top-level
    DG) and a moving jump through outflow x and z boundaries on 4x2x2 K = 8 elements;
    and 40 SSP-RK(5,4) steps of the K = 8 shear layer.
    State within 1e-9, step sizes within 1e-11 (the oracle's own trajectories move by
    at most 1.2e-13 under a 1e-15 relative perturbation of their initial states)."""
    if case.startswith("shear"):
        ne, K = (4, 4) if "K4" in case else (2, 8)
        mesh, u, _ = W.shear_layer_3d(0, ne, K)
        u = u.numpy()
    else:
        mesh, u = _jump_3d(8, [4, 2, 2])
    p = W.Params(cfl=0.5, integrator=sedg.SEDG_SSPRK54 if "RK(5,4)" in case else sedg.SEDG_SSPRK3)
    u_o, dts_o = O.rk3(mesh, p, u, steps)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(np.ascontiguousarray(u)).to(DEV)
    dts = torch.zeros(steps, dtype=torch.float64, device=DEV)
    s.rk_step(ug, steps, 0.0, dts)
    s.check()
    err = rel_err(ug.cpu().numpy(), u_o)
    dterr = np.abs(dts.cpu().numpy() - dts_o).max() / dts_o.max()
    _, info = O.rhs(mesh, p, u_o, full=True)
    nb = int((info["alpha"][:, 0] < 1.0).sum())
    say("  rk3 3-D %s %d steps rel_err=%.3e dt_err=%.3e; at the end %d of %d elements below pure top-level DG"
        % (case, steps, err, dterr, nb, mesh.nel))
    if "K8" in case:
        assert nb > 0
    assert err <= STATE_TOL and dterr <= 1e-11
    s.close()


def test_rk3_fixed_dt_and_repeat_bitwise():
    mesh, u, _ = W.config0(1, 8, 8)
    p = W.Params()
    outs = []
    for _ in range(2):
        s = sedg.Solver(mesh, p)
        ug = torch.from_numpy(u).to(DEV)
        s.rk_step(ug, 5, 1e-4)
        s.check()
        outs.append(ug.cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])
    u_o, _ = O.rk3(mesh, p, u, 5, 1e-4)
    assert rel_err(outs[0], u_o) <= STATE_TOL


def test_max_dt():
    mesh, u, _ = W.sedov(0, 16, 8)
    p = W.Params(cfl=0.5)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u).to(DEV)
    d = torch.zeros(1, dtype=torch.float64, device=DEV)
    s.max_dt(ug, d)
    s.check()
    assert abs(d.item() - O.max_dt(mesh, p, u)) <= 1e-15 * d.item()
    s.close()


def _one_ulp_change(wm, p, sub, do, sel):
    """The oracle's own largest change of its right-hand side over sel when its input moves
    by one ulp (relative, random signs): the FP64 conditioning of the window."""
    noise = 0.0
    for t in range(2):
        sgn = np.random.default_rng(100 + t).choice([-1.0, 1.0], size=sub.shape)
        dp = O.rhs(wm, p, np.ascontiguousarray(sub * (1.0 + sgn * 2.220446049250313e-16)))
        noise = max(noise, np.abs(dp - do)[sel].max())
    return noise


def _window_compare(label, go, oo, noise):
    """Bar: 1e-12 of the window's largest right-hand side, or 4 times the oracle's own
    1-ulp change where that is larger; both are printed."""
    scale = np.abs(oo).max()
    err = np.abs(go - oo).max()
    bar = RHS_TOL * scale
    tol = max(bar, 4.0 * noise)
    say("  %s |g-o|=%.3e  max|o|=%.3e  rel=%.3e  (1e-12 bar %.3e; oracle 1-ulp change %.3e: %s)"
        % (label, err, scale, err / scale, bar, noise,
           "within the 1e-12 bar" if err <= bar else "above the 1e-12 bar, within 4x the 1-ulp change"))
    assert err <= tol
    return err / scale


def _full_size_blast(steps):
    mesh, u, info = W.sedov(0, 256, 8)
    p = W.Params()
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u).to(DEV)
    if steps:
        s.rk_step(ug, steps)
        s.check()
    dg = torch.zeros_like(ug)
    A = W.alpha_len(mesh, p)
    al = torch.zeros(mesh.nel * A, dtype=torch.float64, device=DEV)
    be = torch.zeros_like(al)
    s.rhs(ug, dg, al, be)
    s.check()
    out = (mesh, p, ug.cpu().numpy(), dg.cpu().numpy(), al.cpu().numpy().reshape(mesh.nel, A),
           be.cpu().numpy().reshape(mesh.nel, A), s, ug)
    return out


@pytest.mark.parametrize("steps", [0, 200, 1000])
def test_full_size_sedov_windows(steps):
    """256x256 elements, K = 8 (the benchmark's launch configuration), at the initial
    state and after 200 and 1000 GPU steps (the state handed to the oracle): the right-hand side
    of 5x5-element windows on the blast (its centre, its flanks and, after 200 steps,
    elements whose top level is blended or rejected, where there are any) equals the
    oracle's on the window (interior 3x3 elements; factors and face states are
    element-local)."""
    mesh, p, u, d, al, be, s, ug = _full_size_blast(steps)
    K, ne = 8, 256
    A = al.shape[1]
    aln, ben = al.reshape(ne, ne, A), be.reshape(ne, ne, A)
    # the element holding the blast centre
    c = W.sedov(0, 256, 8)[2]["center"]
    cx, cy = int((c[0] + 1.5) / (3.0 / ne)), int((c[1] + 1.5) / (3.0 / ne))
    # the centre, the flanks at 5 and 12 elements and a diagonal at 9 (the Gaussian's
    # width is 5 elements: its steepest pressure gradient lies near 5, its tail beyond)
    centres = [(cx, cy), (cx + 5, cy), (cx, cy - 12), (cx - 9, cy + 9)]
    # elements whose top-level factor is below 1 (blended or rejected), if any
    front = np.argwhere(aln[:, :, 0] < 1.0)
    say("  step %d: %d elements below pure top-level DG, %d squeezed sub-elements"
        % (steps, len(front), int((be < 1.0).sum())))
    if len(front):
        rng = np.random.default_rng(7)
        pick = front[rng.choice(len(front), size=min(4, len(front)), replace=False)]
        centres += [(int(x), int(y)) for y, x in pick if 2 <= x < ne - 2 and 2 <= y < ne - 2]
    rels = []
    for (ex, ey) in centres:
        x0, y0 = ex - 2, ey - 2
        assert 0 <= x0 and x0 + 5 <= ne and 0 <= y0 and y0 + 5 <= ne
        h = 3.0 / ne
        sub = np.ascontiguousarray(u[:, :, y0 * K:(y0 + 5) * K, x0 * K:(x0 + 5) * K])
        wm = W.Mesh(2, K, [5, 5], [-1.5 + x0 * h, -1.5 + y0 * h], [-1.5 + (x0 + 5) * h, -1.5 + (y0 + 5) * h], [1, 1])
        do, info = O.rhs(wm, p, sub, full=True)
        label = "step %d window (%d,%d)" % (steps, ex, ey)
        fnoise = factor_noise(wm, p, sub, info)
        exempt = check_factors(np.ascontiguousarray(aln[y0:y0 + 5, x0:x0 + 5].reshape(25, A)),
                               np.ascontiguousarray(ben[y0:y0 + 5, x0:x0 + 5].reshape(25, A)), info, p, label,
                               fnoise)
        go = d[:, :, (y0 + 1) * K:(y0 + 4) * K, (x0 + 1) * K:(x0 + 4) * K]
        if exempt:
            # the oracle's decisions in the window, fed to the GPU (and to the oracle)
            a2 = aln.copy()
            a2[y0:y0 + 5, x0:x0 + 5] = info["alpha"].reshape(5, 5, A)
            pe = W.Params(mode=W.EXTERNAL)
            s2 = sedg.Solver(mesh, pe)
            d2 = torch.zeros_like(ug)
            s2.rhs(ug, d2, None, None, torch.from_numpy(a2.reshape(-1)).to(DEV))
            s2.check()
            s2.close()
            go = d2.cpu().numpy()[:, :, (y0 + 1) * K:(y0 + 4) * K, (x0 + 1) * K:(x0 + 4) * K]
            do = O.rhs(wm, pe, sub, alpha_in=info["alpha"])
        oo = do[:, :, K:4 * K, K:4 * K]
        n_blend = int(((info["alpha"][:, 0] > 0) & (info["alpha"][:, 0] < 1)).sum())
        n_sq = int((info["beta"] < 1.0).sum())
        say("  %s: %d blended top-level factors, %d squeezed sub-elements, %d fallbacks, %d exempt, "
            "oracle 1-ulp change of its factors %.1e" % (label, n_blend, n_sq, info["fallbacks"], len(exempt), fnoise))
        # every window lies on the blast: its right-hand side is far above rounding noise
        assert np.abs(oo).max() > 1e-6
        sel = (slice(None), slice(None), slice(K, 4 * K), slice(K, 4 * K))
        d_ad = do if not exempt else O.rhs(wm, p, sub)
        rels.append(_window_compare(label, go, oo, _one_ulp_change(wm, p, sub, d_ad, sel)))
    s.close()
    say("  step %d: largest window error %.3e of max|o|" % (steps, max(rels)))


def test_full_size_shear3d_windows():
    """64^3 elements, K = 8 (the 3-D benchmark's launch configuration): the right-hand
    side of sampled 3x3x3-element windows equals the oracle's on the window cut out with
    one ring of neighbours (outflow edges on the cut, interior compared), at windows on
    the two shear layers (y = -1/2, +1/2), on the mid-plane and at seeded positions."""
    mesh, ud, _ = W.shear_layer_3d(0, 64, 8, nq=3, device=DEV)
    p = W.Params()
    s = sedg.Solver(mesh, p)
    ug = ud.contiguous()
    del ud
    dg = torch.zeros_like(ug)
    s.rhs(ug, dg)
    s.check()
    s.close()
    K, ne, h = 8, 64, 2.0 / 64
    rng = np.random.default_rng(5)
    centres = [(10, 16, 20), (40, 48, 33), (31, 32, 31), (5, 15, 58)]
    centres += [(int(rng.integers(2, 62)), int(rng.choice([15, 16, 47, 48])), int(rng.integers(2, 62))) for _ in range(2)]
    for (ex, ey, ez) in centres:
        x0, y0, z0 = ex - 2, ey - 2, ez - 2
        sub = np.ascontiguousarray(ug[:, z0 * K:(z0 + 5) * K, y0 * K:(y0 + 5) * K, x0 * K:(x0 + 5) * K].cpu().numpy())
        wm = W.Mesh(3, K, [5, 5, 5], [-1.0 + x0 * h, -1.0 + y0 * h, -1.0 + z0 * h],
                    [-1.0 + (x0 + 5) * h, -1.0 + (y0 + 5) * h, -1.0 + (z0 + 5) * h], [1, 1, 1])
        do = O.rhs(wm, p, sub)
        go = dg[:, (z0 + 1) * K:(z0 + 4) * K, (y0 + 1) * K:(y0 + 4) * K, (x0 + 1) * K:(x0 + 4) * K].cpu().numpy()
        oo = do[:, K:4 * K, K:4 * K, K:4 * K]
        noise = _one_ulp_change(wm, p, sub, do, (slice(None), slice(K, 4 * K), slice(K, 4 * K), slice(K, 4 * K)))
        _window_compare("3-D window (%d,%d,%d)" % (ex, ey, ez), go, oo, noise)
    del ug, dg
    torch.cuda.empty_cache()


def test_full_size_conservation_periodic():
    """128x128 elements, K = 8, periodic: the domain sum of the right-hand side
    vanishes to round-off for adaptive and random blending factors."""
    mesh, u, _ = W.pressure_pulse(0, 128, 8)
    for mode in (W.ADAPTIVE, W.EXTERNAL):
        p = W.Params(mode=mode)
        al = None
        if mode == W.EXTERNAL:
            al = np.random.default_rng(1).uniform(0, 1, size=(mesh.nel, W.alpha_len(mesh, p)))
        d, _, _ = gpu_rhs(mesh, p, u, al)
        tot = d.reshape(4, -1).sum(1)
        scale = np.abs(d).reshape(4, -1).sum(1)
        say("  conservation mode%d rel=%s" % (mode, (np.abs(tot) / scale)))
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_free_stream_gpu():
    mesh = W.Mesh(2, 8, [9, 7], [0, 0], [1, 1], [0, 0])
    u = np.zeros(mesh.shape())
    u[0], u[1], u[2], u[3] = 1.3, 0.4, -0.25, 3.0
    p = W.Params(mode=W.EXTERNAL)
    al = np.random.default_rng(2).uniform(0, 1, size=(mesh.nel, W.alpha_len(mesh, p)))
    d, _, _ = gpu_rhs(mesh, p, u, al)
    assert np.abs(d).max() <= 1e-13 * 10 * 8 * 9


def test_bad_state_reported():
    """A negative density is reported by sedg_check with its element; the kernels
    finish normally."""
    mesh, u, _ = W.config0(0, 8, 4)
    u = u.copy()
    u[0, 0, 13, 9] = -1.0     # subcell (9, 13) lies in element (2, 3) = 2 + 8 * 3
    s = sedg.Solver(mesh, W.Params())
    ug = torch.from_numpy(u).to(DEV)
    dg = torch.zeros_like(ug)
    s.rhs(ug, dg)
    with pytest.raises(sedg.SedgError) as ei:
        s.check()
    assert ei.value.code == sedg.SEDG_ESTATE and "element 26" in str(ei.value)
    assert s.check() == -1     # flag cleared
    s.close()


def test_invalid_arguments():
    mesh, u, _ = W.config0(0, 4, 4)
    with pytest.raises(sedg.SedgError):
        sedg.Solver(W.Mesh(2, 6, [2, 2], [0, 0], [1, 1], [0, 0]), W.Params())
    with pytest.raises(sedg.SedgError):
        sedg.Solver(mesh, W.Params(top_level=3))
    s = sedg.Solver(mesh, W.Params(mode=W.EXTERNAL))
    ug = torch.from_numpy(u).to(DEV)
    with pytest.raises(sedg.SedgError):
        s.rhs(ug, torch.zeros_like(ug))        # EXTERNAL without alpha_in
    with pytest.raises(sedg.SedgError):
        s.rk_step(ug, 1)                        # EXTERNAL cannot step
    s.close()
    s = sedg.Solver(mesh, W.Params())
    with pytest.raises(sedg.SedgError) as ei:
        s.rhs(ug, ug)                           # the output may not alias the state
    assert ei.value.code == sedg.SEDG_EINVAL
    with pytest.raises(sedg.SedgError) as ei:
        s.rk_step(ug, -1)
    assert ei.value.code == sedg.SEDG_EINVAL
    before = ug.clone()
    s.rk_step(ug, 0)                            # zero steps: nothing happens
    assert torch.equal(ug, before)
    s.close()
