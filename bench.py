#!/usr/bin/env python3
"""Benchmark: FP64 DOF-updates per second of the sub-element adaptive blended
DG/FV scheme with SSP-RK3 on one MI355X.

Workload (the configuration the metric is quoted on): 2-D Sedov-type blast,
256 x 256 Cartesian elements over [-1.5, 1.5]^2 with outflow boundaries,
K = 8 mean values per direction (polynomial degree 7, hierarchy O(8) -> O(4)
-> O(2) -> FV), FP64, CFL 0.5, synthetic seeded initial state (background
rho = 1, p = 1e-5, v = 0; blast energy 1 deposited as a Gaussian of width 0.06
at a seeded centre within 0.1 of the origin).

One step = one SSP-RK3 step = 3 right-hand-side evaluations with their stage
updates.  value = DOF x 3 x steps / time, DOF = subcell mean values
(4,194,304).  The timed region is the whole configured run, 1000 steps from the
initial state (warm-up steps run on a scratch copy first), as the library runs it:
one HIP graph replay per step, nothing else on the stream.  A second run of the same
steps, launched directly with one HIP event at every launch boundary on the
library's stream, gives the per-kernel durations of the roofline figure.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per DOF and SSP-RK3 stage of the fused stage: state I/O (read
# the stage state, read u^n in two of three stages, write the next state) plus one write
# and one read of the exchanged face states and factors, averaged over the three stages
STAGE_BYTES_PER_DOF = {(2, 8): 123.0, (2, 4): 154.0, (3, 8): 169.0}
METRIC = "FP64 DOF-updates/sec on 1 MI355X (fwd, batched, adjoint/fwd cost ratio)"


def kernel_bytes_per_launch(mesh, A):
    """Algorithmic HBM bytes of one launch of each stage kernel (minimal I/O of the
    decomposition): the analysis (state in; factors, face states and scales out), the
    element-face fluxes and the residual (state in and out, stage base state, own
    factors, element-face fluxes, scales).  The sub-element means travel only for
    squeezed sub-elements (they enter only as (1 - beta) <u>), none in this count."""
    d, K, nv = mesh.dim, mesh.K, mesh.nvar
    nel = mesh.nel
    kd, kf = K ** d, K ** (d - 1)
    per_el = {
        "analyse": 8 * (nv * kd + 2 * A + 2 * d * nv * kf + 2),
        # element-face fluxes, once per face: the element's d low faces (face states of
        # both sides, both elements' factors and scales in; F* out)
        "faces": 8 * (d * (2 * nv * kf + 2 * A + 4) + d * nv * kf),
        # state in, out, stage base state (2 of 3 stages), own factors, the fluxes on
        # its 2d element faces, own scales
        "residual": 8 * (nv * kd + nv * kd + (2.0 / 3.0) * nv * kd + 2 * A + 2 * d * nv * kf + 2),
    }
    return {k: v * nel for k, v in per_el.items()}


KERNEL_SRC = os.path.join(ROOT, "paper_2011_03338_amd", "csrc", "sedg_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernels_sedov2d_256x256_K8_hbm_traffic.txt")


def kernel_source_sha1():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when
    the summary is missing, covers another kernel, or the kernel source changed
    since the counters were taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha1") != kernel_source_sha1():
            return None
        return float(kv["%s_hbm_bytes_per_launch" % kernel])
    except (OSError, KeyError, ValueError):
        return None


def measured_stage_traffic():
    """HBM bytes of one stage (analyse + element faces + residual launches) from the
    committed counter summary, or None (see measured_traffic)."""
    parts = [measured_traffic(k) for k in ("analyse", "faces", "residual")]
    return None if any(x is None for x in parts) else sum(parts)


def copy_probe(mib, dev):
    """A plain device copy of known size (mib MiB read, mib MiB written), for
    calibrating the HBM byte counters; untimed."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def copy_bandwidth(dev, mib=2048, reps=10):
    """Achieved HBM bandwidth of a plain device-to-device copy (mib MiB read and mib MiB
    written per copy), the practical ceiling beside the 8 TB/s nominal peak."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"bytes_per_copy": 2 * mib * (1 << 20), "ms": ms, "GBs": 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9}


def cpu_baseline(mesh, params, u, min_seconds=10.0, max_seconds=30.0):
    """The oracle (plain FP64 C, OpenMP over elements) on the host cores: whole
    SSP-RK3 steps of the same workload from its initial state until at least
    min_seconds of work (stopping before max_seconds would be exceeded)."""
    from oracle import oracle as O
    x, steps, spent = u, 0, 0.0
    while spent < min_seconds:
        t0 = time.perf_counter()
        x, _ = O.rk3(mesh, params, x, 1)
        spent += time.perf_counter() - t0
        steps += 1
        if spent + spent / steps > max_seconds:
            break
    return {"value": mesh.dof * 3 * steps / spent, "unit": "DOF-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "%d SSP-RK3 step(s) (3 right-hand sides each) of the full 256x256-element K=8 blast from "
                      "its initial state, %.1f s" % (steps, spent)}


def adjoint_bench(args, dev):
    """Adjoint workload: 2-D Euler, 128x128 periodic elements over [0,1]^2, K = 8;
    config-0 state plus a Gaussian pressure pulse (amplitude 5, width 0.05).
    J = sum of rho^2 |cell| over the cells centred in [0.4, 0.6]^2 after `adj_steps`
    SSP-RK3 steps (CFL 0.5); gradient with respect to the initial state through the
    checkpointed autograd evolution (checkpoint every 20 steps, frozen factors and
    step sizes).  Reports the forward time, the backward time (replay of every
    segment from its checkpoint plus the transposed steps) and their ratio, and
    central differences of the frozen map along seeded unit directions.  The
    difference error is truncation-dominated at steps of 1e-6 |u0| (the frozen map
    has kinks where Einfeldt speed estimates tie) and rounding-dominated below
    1e-9 |u0|; 1e-7 |u0| sits between the two."""
    import numpy as np
    import torch
    from paper_2011_03338_amd import adjoint as ADJ, sedg, workloads as W
    mesh, u0n, info = W.pressure_pulse(args.seed, 128, 8)
    s = sedg.Solver(mesh, W.Params(cfl=0.5))
    u0 = torch.from_numpy(u0n).to(dev).reshape(-1)
    G = mesh.grid
    xc = (np.arange(G[0]) + 0.5) / G[0]
    yc = (np.arange(G[1]) + 0.5) / G[1]
    win = torch.from_numpy(((yc[:, None] >= 0.4) & (yc[:, None] <= 0.6) &
                            (xc[None, :] >= 0.4) & (xc[None, :] <= 0.6)).astype(np.float64)).to(dev)
    cell = 1.0 / (G[0] * G[1])

    def J(u):
        return (u[:G[0] * G[1]].reshape(G[1], G[0]) ** 2 * win).sum() * cell

    x = u0.clone().requires_grad_(True)
    J(ADJ.evolve(x, s, 3, 20)).backward()           # warm-up: graph capture, buffers
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    x = u0.clone().requires_grad_(True)
    ev[0].record()
    uT = ADJ.evolve(x, s, args.adj_steps, 20)
    jv = J(uT)
    ev[1].record()
    jv.backward()
    ev[2].record()
    torch.cuda.synchronize()
    fwd_ms, bwd_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    grad = x.grad.detach()
    fd = None
    if args.adj_fd > 0:
        dts = ADJ.dt_log_of(uT)[:args.adj_steps].clone()
        frozen = ADJ.record_frozen(s, u0, dts)
        dirs = []
        rng = np.random.default_rng(args.seed + 1000)
        for _ in range(args.adj_fd):
            v = torch.from_numpy(rng.standard_normal(u0.numel())).to(dev)
            dirs.append(v / v.norm())
        ads = [float((grad * v).sum()) for v in dirs]
        # second measure: errors relative to the root mean square of the directional
        # derivatives, which does not blow up on a direction nearly orthogonal to the gradient
        rms = float(np.sqrt(np.mean(np.square(ads))))

        def central(eps):
            errs, abserrs = [], []
            for v, ad in zip(dirs, ads):
                jp = J(ADJ.frozen_evolve(s, u0 + eps * v, frozen, dts))
                jm = J(ADJ.frozen_evolve(s, u0 - eps * v, frozen, dts))
                fdv = float((jp - jm) / (2 * eps))
                errs.append(abs(fdv - ad) / max(abs(ad), 1e-300))
                abserrs.append(abs(fdv - ad))
            return {"eps": eps, "max_rel_err": max(errs), "n_within_1e-6": int(sum(e <= 1e-6 for e in errs)),
                    "max_err_rel_to_rms_derivative": max(abserrs) / rms, "rel_errs": errs}

        chosen = central(args.adj_fd_eps * float(u0.norm()))
        fd = {"directions": args.adj_fd, "eps_relative_to_norm": args.adj_fd_eps, "max_rel_err": chosen["max_rel_err"],
              "within_1e-6": chosen["max_rel_err"] <= 1e-6, "n_within_1e-6": chosen["n_within_1e-6"],
              "max_err_rel_to_rms_derivative": chosen["max_err_rel_to_rms_derivative"],
              "rel_errs": chosen["rel_errs"], "directional_derivatives": ads,
              # the workload's configured step 1e-6, read as absolute and as relative to |u0|
              "configured_eps_1e-6_absolute": central(1e-6),
              "configured_eps_1e-6_relative_to_norm": central(1e-6 * float(u0.norm()))}
    s.check()
    dof = mesh.dof
    return {"workload": "2-D Euler pressure pulse, 128x128 periodic elements, K=8, %d SSP-RK3 steps, "
                        "checkpoint every 20" % args.adj_steps,
            "J": float(jv.detach()), "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "adjoint_fwd_cost_ratio": bwd_ms / fwd_ms,
            "fwd_dof_updates_per_s": dof * 3 * args.adj_steps / (fwd_ms * 1e-3),
            "finite_differences": fd, "pulse_center": info["pulse_center"]}


def fwd3d_bench(args, dev):
    """3-D forward: Kelvin-Helmholtz shear layer, 64^3 periodic elements over [-1, 1]^3,
    K = 8 (degree 7, O(8) -> O(4) -> O(2) -> FV), 134 M DOF, CFL 0.5; means of the
    initial state by a 3^3 Gauss rule per subcell, computed on the GPU; `steps3d`
    timed SSP-RK3 steps after one warm-up step, with per-launch events."""
    import torch
    from paper_2011_03338_amd import sedg, workloads as W
    mesh, u0, _ = W.shear_layer_3d(args.seed, 64, 8, nq=3, device="cuda")
    params = W.Params(cfl=0.5)
    s = sedg.Solver(mesh, params)
    u = u0.contiguous().reshape(-1)
    del u0
    s.rk_step(u, 1)
    s.check()
    s.profile(True)
    s.profile_read()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.rk_step(u, args.steps3d)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = s.profile_read()
    s.profile(False)
    s.check()
    kb = kernel_bytes_per_launch(mesh, W.alpha_len(mesh, params))
    kernels = {k: {"avg_ms": (prof[k][0] / prof[k][1]) if prof[k][1] else None, "launches": prof[k][1],
                   "algorithmic_GBs": (kb[k] / ((prof[k][0] / prof[k][1]) * 1e-3) / 1e9) if k in kb and prof[k][1] else None}
               for k in prof}
    stage_ms = sum(kernels[k]["avg_ms"] for k in ("analyse", "faces", "residual")) + \
        (prof["step_size"][0] / max(prof["step_size"][1], 1)) / 3.0
    stage_gbs = STAGE_BYTES_PER_DOF[(3, 8)] * mesh.dof / (stage_ms * 1e-3) / 1e9
    s.close()
    return {"workload": "3-D Kelvin-Helmholtz shear layer, 64^3 periodic elements, K=8, SSP-RK3 CFL 0.5",
            "value": mesh.dof * 3 * args.steps3d / (ms * 1e-3), "unit": "DOF-updates/s",
            "steps": args.steps3d, "ms_per_step": ms / args.steps3d, "dof": mesh.dof, "kernels": kernels,
            "stage_ms": stage_ms, "stage_algorithmic_GBs": stage_gbs, "stage_frac_of_hbm": stage_gbs / HBM_PEAK_GBS}


def batch_bench(args, dev, steps=None, sigma_floor=0.0):
    """Batched ensemble: 256 independent 2-D Sedov-type blasts ([-1.5, 1.5]^2,
    outflow), mesh side drawn from {32, 48, 64, 96, 128} elements, K from {4, 8},
    blast energy in [0.5, 2], centre within 0.2 of the origin, each with its own CFL
    step; `batch_steps` (default 50) SSP-RK3 steps of the whole ensemble, one analyse and one
    residual launch per stage, the step captured in a HIP graph; launch shape from
    the autotuner (timed outside the measured region)."""
    import torch
    from paper_2011_03338_amd import autotune, sedg, workloads as W
    descs = W.ensemble(args.seed, 256)
    meshes, states = [], []
    for d in descs:
        m, x, _ = W.ensemble_problem(d)
        meshes.append(m)
        states.append(x)
    steps = args.batch_steps if steps is None else steps
    B = sedg.BatchSolver(meshes, W.Params(cfl=0.5, sigma_floor=sigma_floor))
    u = B.pack(states)
    del states
    tuning, timings, cached = autotune.tune(B, u, steps=2)
    B.rk_step(u, 1)                                  # warm-up (graph capture)
    B.check()
    log = torch.zeros(steps * B.count, dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    B.rk_step(u, steps, 0.0, log)
    ev1.record()
    torch.cuda.synchronize()
    B.check()
    ms = ev0.elapsed_time(ev1)
    dof = sum(m.dof for m in meshes)
    nbytes = 0.0
    for m in meshes:
        kb = kernel_bytes_per_launch(m, W.alpha_len(m, W.Params()))
        nbytes += kb["analyse"] + kb["residual"]
    gbs = nbytes * 3 * steps / (ms * 1e-3) / 1e9
    ks = {}
    for m in meshes:
        ks.setdefault(m.K, [0, 0])
        ks[m.K][0] += 1
        ks[m.K][1] += m.dof
    return {"workload": "256 independent 2-D Sedov blasts, sides {32..128}^2 elements, K in {4,8}, "
                        "per-problem CFL 0.5, %d SSP-RK3 steps%s"
                        % (steps, "" if sigma_floor <= 0 else
                           ", indicator denominator floor %g (a variant; the paper's floor is 1)" % sigma_floor),
            "value": dof * 3 * steps / (ms * 1e-3), "unit": "DOF-updates/s",
            "ms_per_step": ms / steps, "problems": B.count, "dof": dof,
            "problems_dof_by_K": {str(k): v for k, v in sorted(ks.items())},
            "tuning": tuning, "tuning_from_cache": cached,
            "tuning_ms_per_step": {str(k): v for k, v in timings.items()},
            "algorithmic_GBs": gbs, "algorithmic_frac_of_hbm": gbs / HBM_PEAK_GBS,
            "dt_log_finite": bool(torch.isfinite(log).all().item()),
            "dt_range": [float(log.min()), float(log.max())]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--adj-fd", type=int, default=32, help="finite-difference directions of the adjoint check")
    ap.add_argument("--adj-fd-eps", type=float, default=1e-7,
                    help="central-difference step along unit directions, relative to the initial state's norm")
    ap.add_argument("--no-adjoint", action="store_true")
    # 50: every member stays permissible; 25 of the 31 members with 32^2 elements at
    # K = 8 lose positivity between steps 55 and 100 (the oracle too)
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--steps3d", type=int, default=5)
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run an untimed device copy of this size first (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single MI355X "
              "(sharding over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2011_03338_amd import sedg, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib, dev)
    mesh, u0, info = W.sedov(args.seed, 256, 8)
    params = W.Params(cfl=0.5)
    A = W.alpha_len(mesh, params)
    s = sedg.Solver(mesh, params)
    u = torch.from_numpy(u0).to(dev)
    stream = torch.cuda.current_stream()

    # warm-up on a scratch copy (graph capture, first launches of both launch paths); the
    # timed run starts from the initial state
    uw = u.clone()
    s.rk_step(uw, args.warmup)
    s.profile(True)
    s.rk_step(uw, 1)
    s.profile_read()
    s.profile(False)
    s.check()
    del uw
    torch.cuda.synchronize()

    # timed region: the whole run as the library runs it (one HIP graph replay per step),
    # with no instrumentation inside
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.rk_step(u, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s.check()
    dof = mesh.dof
    value = dof * 3 * args.steps / (ms * 1e-3)

    # the same run again from the initial state, launched directly with one HIP event at
    # every launch boundary on the library's stream: the per-kernel durations of the
    # roofline (the events add a little time between launches, so this run is slower)
    up = torch.from_numpy(u0).to(dev)
    s.profile(True)
    ev0.record(stream)
    s.rk_step(up, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_profiled = ev0.elapsed_time(ev1)
    prof = s.profile_read()
    s.profile(False)
    s.check()
    same_state = bool(torch.equal(up, u))
    del up

    # roofline: one stage (analyse + element faces + residual; a separate step-size kernel,
    # where one runs, counted once per three stages) against the algorithmic bytes of a
    # fused stage
    kb = kernel_bytes_per_launch(mesh, A)
    kernels = {k: {"avg_ms": (prof[k][0] / prof[k][1]) if prof[k][1] else None, "launches": prof[k][1],
                   "algorithmic_GBs": (kb[k] / ((prof[k][0] / prof[k][1]) * 1e-3) / 1e9) if k in kb and prof[k][1] else None}
               for k in prof}
    stage_ms = sum(kernels[k]["avg_ms"] for k in ("analyse", "faces", "residual")) + \
        (prof["step_size"][0] / max(prof["step_size"][1], 1)) / 3.0
    stage_bytes = STAGE_BYTES_PER_DOF[(mesh.dim, mesh.K)] * dof
    achieved = stage_bytes / (stage_ms * 1e-3) / 1e9
    traffic = measured_stage_traffic()
    copy_bw = copy_bandwidth(dev)
    roof = {"bound": "hbm", "kernel": "SSP-RK3 stage: analyse + element faces + residual (the step size is formed inside the first stage's element-face launch)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "algorithmic_bytes_per_stage": stage_bytes,
            "algorithmic_bytes_per_dof_stage": STAGE_BYTES_PER_DOF[(mesh.dim, mesh.K)],
            "avg_stage_ms": stage_ms, "dof_per_stage": dof,
            "traffic_over_algorithmic": (traffic / stage_bytes) if traffic else None,
            "dominant_kernel": max(("analyse", "residual", "faces"), key=lambda k: prof[k][0]),
            "device_copy": copy_bw, "frac_of_device_copy": achieved / copy_bw["GBs"]}

    # activity of the scheme over the same run (untimed, from the initial state again):
    # the right-hand-side diagnostics every 100 steps
    activity = []
    ua = torch.from_numpy(u0).to(dev)
    da = torch.zeros_like(ua)
    done = 0
    while True:
        dg = s.diagnose(ua, da)
        activity.append({"step": done, "elements_by_lowest_order": dg["elems_by_lowest_order"],
                         "squeezed_subelements": dg["squeezed"], "beta_rejected_subelements": dg["beta_rejected"],
                         "interface_fallbacks": dg["fallbacks"], "alpha_bar_mean": dg["alpha_bar_mean"],
                         "alpha_bar_min": dg["alpha_bar_min"]})
        if done >= args.steps:
            break
        m = min(100, args.steps - done)
        s.rk_step(ua, m)
        done += m
    s.check()
    del ua, da

    adj = None if args.no_adjoint else adjoint_bench(args, dev)
    batch = None if args.no_batch else batch_bench(args, dev)
    # the configured 200 steps: with the paper's indicator floor of 1, 25 of the 31 coarse
    # K = 8 members lose positivity between steps 55 and 100 (the oracle alike); with the
    # floor below the data's scale every member stays permissible
    batch200 = None
    if not args.no_batch:
        try:
            batch200 = batch_bench(args, dev, 200, 1e-14)
        except RuntimeError as e:     # a member lost positivity: report it, keep the rest
            batch200 = {"failed": str(e)}
    fwd3d = None if args.no_3d else fwd3d_bench(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, params, u0)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D Sedov blast, 256x256 elements, K=8 (degree 7, O(8)->O(4)->O(2)->FV), "
                               "outflow, SSP-RK3 CFL 0.5, the whole %d-step run from the initial state" % args.steps,
                   "elements": mesh.nel, "K": mesh.K, "dof": dof, "dof_per_var_total": dof * mesh.nvar,
                   "stages_per_step": 3, "blast_center": info["center"]},
        "roofline": roof,
        "kernels": kernels,
        "profiled_run": {"ms_per_step": ms_profiled / args.steps,
                         "launch": "direct launches with one HIP event at every launch boundary (the per-kernel "
                                   "figures); the timed run replays one HIP graph per step",
                         "same_final_state_bitwise": same_state},
        "activity": activity,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "batched": batch,
        "batched_200_steps_floor_variant": batch200,
        "fwd_3d": fwd3d,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
