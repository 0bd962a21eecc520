"""The HIP path on the shock tubes of the 1-D validation runs (Sec. 3.4) at the paper's
resolution (32 elements of 8 subcells), each posed as a strip of 32 x 1 elements: Sod
(final time 0.2) and Lax (0.15) on the oracle's step sizes, the state after 100 steps
within the multi-step bar of the oracle's, the density against the exact Riemann
solution, and the paper's comparison of the multi-level chain with the single-level
scheme; Shu-Osher (1.8) against a 2048-DOF oracle reference."""
import numpy as np
import pytest
import torch

from paper_2011_03338_amd import sedg, workloads as W
from tests.parity import DEV, STATE_TOL, rel_err, say
from tests.test_oracle_sod import exact_density_means, run_to, shu_osher_reference_means

pytestmark = pytest.mark.gpu

# Over the whole run (861 steps with all levels, 834 with one) rounding can tip the
# indicator at the shock differently: the oracle itself, with its initial state perturbed
# by 1e-15 relative (random signs), moves by 1.6e-14 and 1.5e-14 after 100 steps, and at
# the final time by 8.2e-13 (all levels) and 2.3e-9 (one level).  The end-of-run bar is
# the multi-step bar where that sensitivity is below it and 10 times the sensitivity
# otherwise.
END_TOL = {0: 1e-9, 1 << 3: 2.5e-8}


@pytest.fixture(scope="module")
def sod_runs():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    out = {}
    for mask in (0, 1 << 3):
        mesh, u0, info = W.sod_tube(nelem=32, K=8)
        p = W.Params(level_mask=mask)
        dts = []
        u_o = run_to(mesh, p, u0, info["T"], dts)
        out[mask] = (mesh, p, u0, info, dts, u_o)
    return out


@pytest.mark.parametrize("mask", [0, 1 << 3])
def test_sod_gpu_100_steps(sod_runs, mask):
    """mask 0: all levels O(8) -> O(4) -> O(2) -> FV; 1 << 3: single level O(8) -> FV.
    The first 100 of the oracle's step sizes on both sides: states within 1e-9."""
    from oracle import oracle as O
    mesh, p, u0, info, dts, _ = sod_runs[mask]
    u_o = u0
    for dt in dts[:100]:
        u_o, _ = O.rk3(mesh, p, u_o, 1, dt_fixed=dt)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u0).to(DEV)
    for dt in dts[:100]:
        s.rk_step(ug, 1, dt)
    s.check()
    err = rel_err(ug.cpu().numpy(), u_o)
    s.close()
    say("  sod mask %d 100 steps rel_err=%.3e" % (mask, err))
    assert err <= STATE_TOL


def _gpu_final(mesh, p, u0, dts):
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u0).to(DEV)
    for dt in dts:
        s.rk_step(ug, 1, dt)
    s.check()
    u_g = ug.cpu().numpy()
    s.close()
    return u_g


def test_sod_gpu_final_and_multilevel_vs_single_level(sod_runs):
    """Final state (T = 0.2) within END_TOL of the oracle's for both level masks, the
    density L1 error against the exact solution bounded, and the multi-level chain at
    least 20 % more accurate than the single level on the GPU as in the oracle."""
    l1 = {}
    for mask, bound in ((0, 3e-3), (1 << 3, 4e-3)):
        mesh, p, u0, info, dts, u_o = sod_runs[mask]
        u_g = _gpu_final(mesh, p, u0, dts)
        diff = float(np.max(np.abs(u_g - u_o)))
        rho = u_g[0, 0].mean(axis=0)
        l1[mask] = float(np.mean(np.abs(rho - exact_density_means(mesh.edges(0), info["T"]))))
        say("  sod mask %d %d steps max|gpu-oracle|=%.3e density L1 vs exact=%.3e"
            % (mask, len(dts), diff, l1[mask]))
        assert diff < END_TOL[mask]
        assert l1[mask] < bound
    assert l1[0] < 0.8 * l1[1 << 3]


def _oracle_steps(mesh, p, u0, dts):
    from oracle import oracle as O
    u = u0
    for dt in dts:
        u, _ = O.rk3(mesh, p, u, 1, dt_fixed=dt)
    return u


def _gpu_steps(mesh, p, u0, dts):
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u0).to(DEV)
    for dt in dts:
        s.rk_step(ug, 1, dt)
    s.check()
    out = ug.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("mask", [0, 1 << 3])
def test_lax_gpu(mask):
    """Lax tube: 100 steps on the oracle's step sizes within 1e-9, the whole run (T = 0.15)
    with the density's L1 error against the exact solution bounded."""
    mesh, u0, info = W.lax_tube(32, 8)
    p = W.Params(level_mask=mask)
    dts = []
    run_to(mesh, p, u0, info["T"], dts)
    err = rel_err(_gpu_steps(mesh, p, u0, dts[:100]), _oracle_steps(mesh, p, u0, dts[:100]))
    u_g = _gpu_steps(mesh, p, u0, dts)
    ref = exact_density_means(mesh.edges(0), info["T"], left=info["left"], right=info["right"])
    l1 = float(np.mean(np.abs(u_g[0, 0].mean(axis=0) - ref)))
    say("  lax mask %d: 100 steps rel_err=%.3e; %d steps density L1 vs exact=%.3e" % (mask, err, len(dts), l1))
    assert err <= STATE_TOL
    assert l1 < 1.5e-2


@pytest.fixture(scope="module")
def shu_osher_reference():
    runs = {}
    mesh, u0, info = W.shu_osher(256, 8, dim=1)
    runs[(256, 0)] = (mesh, run_to(mesh, W.Params(), u0, info["T"]))
    return shu_osher_reference_means(runs)


def test_shu_osher_gpu(shu_osher_reference):
    """Shu-Osher tube on the GPU (strip of 32 x 1 elements, CFL steps of the library):
    the state within 1e-9 of the oracle's on the same step sizes after 100 steps (all
    levels) and 10 steps (single level: there the oracle's own trajectory moves by 4e-11
    at step 12 and 1e-9 at step 16 under a 1e-15 relative perturbation of its initial
    state, as indicator decisions at the shock flip; all levels stay below 1e-12 for 100
    steps), and at T = 1.8 the multi-level chain closer to the 2048-DOF oracle reference
    than the single level, overall and in the smooth parts behind the shock (Sec. 3.4)."""
    mesh, u0, info = W.shu_osher(32, 8)
    xc = 0.5 * (mesh.edges(0)[1:] + mesh.edges(0)[:-1])
    smooth = (xc > -3.5) & (xc < 1.5)
    l1 = {}
    for mask in (0, 1 << 3):
        p = W.Params(level_mask=mask)
        s = sedg.Solver(mesh, p)
        ug = torch.from_numpy(u0).to(DEV)
        nst = 100 if mask == 0 else 10
        log = torch.zeros(nst, dtype=torch.float64, device=DEV)
        s.rk_step(ug, nst, 0.0, log)
        s.check()
        err = rel_err(ug.cpu().numpy(), _oracle_steps(mesh, p, u0, log.cpu().numpy()))
        # the rest of the run to T with the library's CFL steps, the last one cut to land on T
        t = float(log.sum())
        dt = torch.zeros(1, dtype=torch.float64, device=DEV)
        while info["T"] - t > 1e-15:
            s.max_dt(ug, dt)
            step = min(float(dt.item()), info["T"] - t)
            s.rk_step(ug, 1, step)
            t += step
        s.check()
        rho = ug.cpu().numpy()[0, 0].mean(axis=0)
        s.close()
        d = np.abs(rho - shu_osher_reference)
        l1[mask] = (float(d.mean()), float(d[smooth].mean()))
        say("  shu-osher mask %d: %d steps rel_err=%.3e; T=1.8 density L1 vs reference %.4f (smooth parts %.4f)"
            % (mask, nst, err, l1[mask][0], l1[mask][1]))
        assert err <= STATE_TOL
    assert l1[0][0] < 0.8 * l1[1 << 3][0] and l1[0][1] < 0.8 * l1[1 << 3][1]
