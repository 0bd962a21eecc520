"""Batched ensembles: many independent 2-D problems (mixed K, mesh sizes and
boundary conditions) advanced by one launch per kernel and stage must give, for
every problem, launch shape and integrator (SSP-RK3, SSP-RK(5,4)), bit for bit the
states and step sizes of the single-problem path (the same element arithmetic), and
match the oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_03338_amd import sedg, workloads as W
from tests.parity import DEV, STATE_TOL, rel_err, say

pytestmark = pytest.mark.gpu

TUNINGS = [dict(epb4=4, epb8=1, blocks_per_cu=0, xcd_map=1), dict(epb4=4, epb8=1, blocks_per_cu=0, xcd_map=0),
           dict(epb4=8, epb8=2, blocks_per_cu=0, xcd_map=1), dict(epb4=4, epb8=1, blocks_per_cu=2, xcd_map=1),
           dict(epb4=8, epb8=2, blocks_per_cu=1, xcd_map=0),
           dict(epb4=4, epb8=1, blocks_per_cu=0, xcd_map=1, waves_analyse=4, waves_residual=3),
           dict(epb4=8, epb8=2, blocks_per_cu=0, xcd_map=1, waves_analyse=4, waves_residual=3)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sedg.load()
    yield


def _problems():
    out = []
    out.append(W.sedov(3, 5, 8, E=1.5, rc=0.2)[:2])
    out.append(W.config0(1, 8, 4)[:2])
    out.append(W.sedov(4, 7, 4, E=0.7, rc=0.2)[:2])
    out.append(W.config0(2, 3, 8)[:2])
    out.append(W.pressure_pulse(2, 4, 8)[:2])
    m = W.Mesh(2, 8, [1, 1], [0, 0], [1, 1], [0, 0])
    out.append((m, W.density_wave(m, vel=(0.3, -0.2, 0), amp=0.2)))
    out.append(W.sedov(5, 6, 4, E=2.0, rc=0.2, L=0.5, sigma=0.05)[:2])
    return out


def _single(mesh, u, nsteps, dt_fixed=0.0):
    s = sedg.Solver(mesh, W.Params())
    ug = torch.from_numpy(np.ascontiguousarray(u)).to(DEV)
    log = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=DEV)
    s.rk_step(ug, nsteps, dt_fixed, None if dt_fixed > 0 else log)
    s.check()
    out = ug.cpu().numpy(), log.cpu().numpy()[:nsteps]
    s.close()
    return out


@pytest.mark.parametrize("tuning", range(len(TUNINGS)))
def test_batch_matches_single_problem_bitwise(tuning):
    probs = _problems()
    nsteps = 3
    B = sedg.BatchSolver([m for m, _ in probs], W.Params())
    B.set_tuning(**TUNINGS[tuning])
    u = B.pack([x for _, x in probs])
    log = torch.zeros(nsteps * B.count, dtype=torch.float64, device=DEV)
    B.rk_step(u, nsteps, 0.0, log)
    B.check()
    logs = log.view(nsteps, B.count).cpu().numpy()
    views = B.views(u)
    for p, (m, x) in enumerate(probs):
        ref, ref_log = _single(m, x, nsteps)
        got = views[p].cpu().numpy()
        assert np.array_equal(got, ref), (tuning, p, np.abs(got - ref).max())
        assert np.array_equal(logs[:, p], ref_log), (tuning, p)
    say("  batch tuning %s: %d problems bitwise equal" % (TUNINGS[tuning], B.count))
    B.close()


def test_batch_fixed_step_bitwise():
    probs = _problems()
    B = sedg.BatchSolver([m for m, _ in probs], W.Params())
    u = B.pack([x for _, x in probs])
    B.rk_step(u, 2, 2e-5)
    B.check()
    views = B.views(u)
    for p, (m, x) in enumerate(probs):
        ref, _ = _single(m, x, 2, 2e-5)
        assert np.array_equal(views[p].cpu().numpy(), ref), p
    B.close()


def test_batch_matches_oracle():
    """Two members after 5 steps against the oracle's own SSP-RK3 (state 1e-9, steps 1e-14)."""
    probs = _problems()
    B = sedg.BatchSolver([m for m, _ in probs], W.Params())
    u = B.pack([x for _, x in probs])
    nsteps = 5
    log = torch.zeros(nsteps * B.count, dtype=torch.float64, device=DEV)
    B.rk_step(u, nsteps, 0.0, log)
    B.check()
    logs = log.view(nsteps, B.count).cpu().numpy()
    views = B.views(u)
    for p in (1, 2):
        m, x = probs[p]
        uo, dto = O.rk3(m, W.Params(), x, nsteps)
        err = rel_err(views[p].cpu().numpy(), uo)
        say("  batch member %d vs oracle after %d steps: rel_err=%.3e" % (p, nsteps, err))
        assert err <= STATE_TOL
        assert np.abs(logs[:, p] - dto).max() <= 1e-14 * dto.max()
    B.close()


@pytest.mark.parametrize("tuning", [0, 3])
def test_batch_rk54_matches_single_problem_bitwise(tuning):
    """SSP-RK(5,4) ensembles (CFL steps, then a fixed step): every member equals the
    single-problem SSP-RK(5,4) path bit for bit, and one member matches the oracle's
    SSP-RK(5,4) (state within the state tolerance, steps within 1e-14)."""
    probs = _problems()
    prm = W.Params(cfl=0.8, integrator=sedg.SEDG_SSPRK54)
    nsteps = 3
    B = sedg.BatchSolver([m for m, _ in probs], prm)
    B.set_tuning(**TUNINGS[tuning])
    u = B.pack([x for _, x in probs])
    log = torch.zeros(nsteps * B.count, dtype=torch.float64, device=DEV)
    B.rk_step(u, nsteps, 0.0, log)
    B.rk_step(u, 1, 1e-5)
    B.check()
    logs = log.view(nsteps, B.count).cpu().numpy()
    views = B.views(u)
    for p, (m, x) in enumerate(probs):
        s = sedg.Solver(m, prm)
        ug = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        rl = torch.zeros(nsteps, dtype=torch.float64, device=DEV)
        s.rk_step(ug, nsteps, 0.0, rl)
        s.rk_step(ug, 1, 1e-5)
        s.check()
        assert np.array_equal(views[p].cpu().numpy(), ug.cpu().numpy()), (tuning, p)
        assert np.array_equal(logs[:, p], rl.cpu().numpy()), (tuning, p)
        s.close()
    m, x = probs[2]
    uo, dto = O.rk3(m, prm, x, nsteps)
    uo, _ = O.rk3(m, prm, uo, 1, dt_fixed=1e-5)
    err = rel_err(views[2].cpu().numpy(), uo)
    say("  batch SSP-RK(5,4), tuning %s: %d problems bitwise equal; member 2 vs oracle rel_err=%.3e"
        % (TUNINGS[tuning], B.count, err))
    assert err <= STATE_TOL and np.abs(logs[:, 2] - dto).max() <= 1e-14 * dto.max()
    B.close()


def test_batch_reports_bad_state():
    probs = _problems()
    # a negative density in element 0 of member 3 (whose elements follow 138 others);
    # within the step the bad state reaches the face neighbours, so the smallest bad
    # element index over the step is that element's
    x = probs[3][1].copy()
    x[0, 0, 3, 5] = -1.0
    probs[3] = (probs[3][0], x)
    B = sedg.BatchSolver([m for m, _ in probs], W.Params())
    u = B.pack([x for _, x in probs])
    B.rk_step(u, 1, 1e-6)
    with pytest.raises(sedg.SedgError) as ei:
        B.check()
    assert ei.value.problem == 3 and ei.value.element == 0
    B.close()


def test_batch_invalid_arguments():
    m2 = W.config0(0, 4, 4)[0]
    m3 = W.Mesh(3, 4, [2, 2, 2], [0.0] * 3, [1.0] * 3, [0, 0, 0])
    with pytest.raises(sedg.SedgError) as ei:
        sedg.BatchSolver([m2, m3], W.Params())
    assert ei.value.code == sedg.SEDG_EUNSUPPORTED
    mg = W.Mesh(2, 4, [4, 4], [0, 0], [1, 1], [0, 0], gamma=1.3)
    with pytest.raises(sedg.SedgError) as ei:
        sedg.BatchSolver([m2, mg], W.Params())
    assert ei.value.code == sedg.SEDG_EINVAL
    B = sedg.BatchSolver([m2], W.Params())
    with pytest.raises(sedg.SedgError):
        B.set_tuning(epb4=8, epb8=1)
    with pytest.raises(sedg.SedgError):
        B.set_tuning(waves_analyse=5)
    with pytest.raises(sedg.SedgError) as ei:
        B.set_tuning(waves_residual=4)
    assert ei.value.code == sedg.SEDG_EUNSUPPORTED
    B.set_tuning(waves_analyse=0, waves_residual=0)
    assert B.get_tuning()["waves_analyse"] == 3 and B.get_tuning()["waves_residual"] == 3
    B.close()


def test_autotuner_picks_and_caches(tmp_path, monkeypatch):
    from paper_2011_03338_amd import autotune
    monkeypatch.setenv("SEDG_TUNING_CACHE", str(tmp_path / "tune.json"))
    probs = _problems()
    B = sedg.BatchSolver([m for m, _ in probs], W.Params())
    u = B.pack([x for _, x in probs])
    u_before = u.clone()
    cands = autotune.CANDIDATES[:3]
    tun, timings, cached = autotune.tune(B, u, steps=1, candidates=cands)
    assert not cached and tun in cands and len(timings) == 3
    assert torch.equal(u, u_before)                  # the state is not advanced
    assert B.get_tuning() == tun
    tun2, _, cached2 = autotune.tune(B, u, steps=1, candidates=cands)
    assert cached2 and tun2 == tun
    B.close()


VARIANTS = [dict(family=W.LGL), dict(mode=W.FORCE_DG), dict(mode=W.FORCE_FV), dict(level_mask=1 << 2),
            dict(family=W.LGL, level_mask=(1 << 3) | (1 << 1))]


@pytest.mark.parametrize("variant", range(len(VARIANTS)))
def test_batch_variants_match_single_problem_bitwise(variant):
    """LGL nodes, forced DG or FV, and reduced level sets: the ensemble path must still
    reproduce the single-problem path bit for bit."""
    import dataclasses
    v = VARIANTS[variant]
    family = v.get("family", W.GAUSS)
    prm = W.Params(**{k: x for k, x in v.items() if k != "family"})
    probs = [(dataclasses.replace(m, family=family), x) for m, x in _problems()]
    if prm.mode == W.FORCE_DG:
        probs = [probs[i] for i in (1, 3, 4, 5)]      # smooth members only
    nsteps = 2
    B = sedg.BatchSolver([m for m, _ in probs], prm)
    u = B.pack([x for _, x in probs])
    log = torch.zeros(nsteps * B.count, dtype=torch.float64, device=DEV)
    B.rk_step(u, nsteps, 0.0, log)
    B.check()
    logs = log.view(nsteps, B.count).cpu().numpy()
    views = B.views(u)
    for p, (m, x) in enumerate(probs):
        s = sedg.Solver(m, prm)
        ug = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        ref_log = torch.zeros(nsteps, dtype=torch.float64, device=DEV)
        s.rk_step(ug, nsteps, 0.0, ref_log)
        s.check()
        assert np.array_equal(views[p].cpu().numpy(), ug.cpu().numpy()), (v, p)
        assert np.array_equal(logs[:, p], ref_log.cpu().numpy()), (v, p)
        s.close()
    say("  batch variant %s: %d problems bitwise equal" % (v, B.count))
    B.close()


def test_full_size_ensemble_members():
    """The benchmark's ensemble (256 blasts, sides {32..128}^2, K in {4, 8}, 74.6 M DOF)
    in two launch shapes: after 2 steps, sampled members equal the single-problem path
    bit for bit (states and step sizes), and a small member matches the oracle."""
    from paper_2011_03338_amd import autotune
    descs = W.ensemble(0, 256)
    meshes, states = [], []
    for d in descs:
        m, x, _ = W.ensemble_problem(d)
        meshes.append(m)
        states.append(x)
    prm = W.Params(cfl=0.5)
    rng = np.random.default_rng(9)
    dofs = np.array([m.dof for m in meshes])
    sample = sorted({int(np.argmax(dofs)), int(np.argmin(dofs))} | {int(i) for i in rng.choice(256, 4, replace=False)})
    nsteps = 2
    for tun in (autotune.CANDIDATES[0], autotune.CANDIDATES[5]):
        B = sedg.BatchSolver(meshes, prm)
        B.set_tuning(**tun)
        u = B.pack(states)
        log = torch.zeros(nsteps * B.count, dtype=torch.float64, device=DEV)
        B.rk_step(u, nsteps, 0.0, log)
        B.check()
        logs = log.view(nsteps, B.count).cpu().numpy()
        views = B.views(u)
        for p in sample:
            s = sedg.Solver(meshes[p], prm)
            ug = torch.from_numpy(np.ascontiguousarray(states[p])).to(DEV)
            rl = torch.zeros(nsteps, dtype=torch.float64, device=DEV)
            s.rk_step(ug, nsteps, 0.0, rl)
            s.check()
            assert np.array_equal(views[p].cpu().numpy(), ug.cpu().numpy()), (tun, p)
            assert np.array_equal(logs[:, p], rl.cpu().numpy()), (tun, p)
            s.close()
        say("  full ensemble, tuning %s: members %s bitwise equal to single solves" % (tun, sample))
        small = int(np.argmin(dofs))
        uo, dto = O.rk3(meshes[small], prm, states[small], nsteps)
        err = rel_err(views[small].cpu().numpy(), uo)
        assert err <= STATE_TOL and np.abs(logs[:, small] - dto).max() <= 1e-14 * dto.max()
        B.close()
        del u
    torch.cuda.empty_cache()
