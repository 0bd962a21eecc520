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
(4,194,304).  The timed region runs the library's kernels with an event pair
around every launch (the same events give the per-kernel durations of the
roofline figure).

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
METRIC = "FP64 DOF-updates/sec on 1 MI355X (fwd, batched, adjoint/fwd cost ratio)"


def kernel_bytes_per_launch(mesh, A):
    """Algorithmic HBM bytes of one launch of each stage kernel (minimal I/O of the
    decomposition): the analysis (state in; factors, sub-element means, face states and
    scales out), the element-face fluxes and the residual (state in and out, stage base
    state, own factors and means, element-face fluxes, scales)."""
    d, K, nv = mesh.dim, mesh.K, mesh.nvar
    nel = mesh.nel
    kd, kf = K ** d, K ** (d - 1)
    per_el = {
        "analyse": 8 * (nv * kd + 2 * A + nv * A + 2 * d * nv * kf + 2),
        # element-face fluxes, once per face: the element's d low faces (face states of
        # both sides, both elements' factors and scales in; F* out)
        "faces": 8 * (d * (2 * nv * kf + 2 * A + 4) + d * nv * kf),
        # state in, out, stage base state (2 of 3 stages), own factors and sub-element
        # means, the fluxes on its 2d element faces, own scales
        "residual": 8 * (nv * kd + nv * kd + (2.0 / 3.0) * nv * kd + 2 * A + nv * A + 2 * d * nv * kf + 2),
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
        rng = np.random.default_rng(args.seed + 1000)
        eps = args.adj_fd_eps * float(u0.norm())
        errs, ads, abserrs = [], [], []
        for _ in range(args.adj_fd):
            v = torch.from_numpy(rng.standard_normal(u0.numel())).to(dev)
            v = v / v.norm()
            jp = J(ADJ.frozen_evolve(s, u0 + eps * v, frozen, dts))
            jm = J(ADJ.frozen_evolve(s, u0 - eps * v, frozen, dts))
            fdv = float((jp - jm) / (2 * eps))
            ad = float((grad * v).sum())
            errs.append(abs(fdv - ad) / max(abs(ad), 1e-300))
            ads.append(ad)
            abserrs.append(abs(fdv - ad))
        # second measure: errors relative to the root mean square of the directional
        # derivatives, which does not blow up on a direction nearly orthogonal to the gradient
        rms = float(np.sqrt(np.mean(np.square(ads))))
        fd = {"directions": args.adj_fd, "eps_relative_to_norm": args.adj_fd_eps, "max_rel_err": max(errs),
              "within_1e-6": max(errs) <= 1e-6, "n_within_1e-6": int(sum(e <= 1e-6 for e in errs)),
              "max_err_rel_to_rms_derivative": max(abserrs) / rms, "rel_errs": errs, "directional_derivatives": ads}
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
    s.close()
    return {"workload": "3-D Kelvin-Helmholtz shear layer, 64^3 periodic elements, K=8, SSP-RK3 CFL 0.5",
            "value": mesh.dof * 3 * args.steps3d / (ms * 1e-3), "unit": "DOF-updates/s",
            "steps": args.steps3d, "ms_per_step": ms / args.steps3d, "dof": mesh.dof, "kernels": kernels}


def batch_bench(args, dev):
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
    B = sedg.BatchSolver(meshes, W.Params(cfl=0.5))
    u = B.pack(states)
    del states
    tuning, timings, cached = autotune.tune(B, u, steps=2)
    B.rk_step(u, 1)                                  # warm-up (graph capture)
    B.check()
    log = torch.zeros(args.batch_steps * B.count, dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    B.rk_step(u, args.batch_steps, 0.0, log)
    ev1.record()
    torch.cuda.synchronize()
    B.check()
    ms = ev0.elapsed_time(ev1)
    dof = sum(m.dof for m in meshes)
    nbytes = 0.0
    for m in meshes:
        kb = kernel_bytes_per_launch(m, W.alpha_len(m, W.Params()))
        nbytes += kb["analyse"] + kb["residual"]
    gbs = nbytes * 3 * args.batch_steps / (ms * 1e-3) / 1e9
    ks = {}
    for m in meshes:
        ks.setdefault(m.K, [0, 0])
        ks[m.K][0] += 1
        ks[m.K][1] += m.dof
    return {"workload": "256 independent 2-D Sedov blasts, sides {32..128}^2 elements, K in {4,8}, "
                        "per-problem CFL 0.5, %d SSP-RK3 steps" % args.batch_steps,
            "value": dof * 3 * args.batch_steps / (ms * 1e-3), "unit": "DOF-updates/s",
            "ms_per_step": ms / args.batch_steps, "problems": B.count, "dof": dof,
            "problems_dof_by_K": {str(k): v for k, v in sorted(ks.items())},
            "tuning": tuning, "tuning_from_cache": cached,
            "tuning_ms_per_step": {str(k): v for k, v in timings.items()},
            "algorithmic_GBs": gbs, "algorithmic_frac_of_hbm": gbs / HBM_PEAK_GBS,
            "dt_log_finite": bool(torch.isfinite(log).all().item()),
            "dt_range": [float(log.min()), float(log.max())]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
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
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path)", file=sys.stderr)
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

    # warm-up (graph replay path)
    s.rk_step(u, args.warmup)
    s.check()
    torch.cuda.synchronize()

    # timed region: per-launch event pairs on the library's stream
    s.profile(True)
    s.profile_read()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.rk_step(u, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = s.profile_read()
    s.profile(False)
    s.check()
    dof = mesh.dof
    value = dof * 3 * args.steps / (ms * 1e-3)

    # roofline of the dominant kernel
    kb = kernel_bytes_per_launch(mesh, A)
    dom = max(("analyse", "residual", "faces"), key=lambda k: prof[k][0])
    avg_ms = prof[dom][0] / max(prof[dom][1], 1)
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
            "algorithmic_bytes_per_launch": kb[dom], "avg_launch_ms": avg_ms}
    kernels = {k: {"avg_ms": (prof[k][0] / prof[k][1]) if prof[k][1] else None, "launches": prof[k][1],
                   "algorithmic_GBs": (kb[k] / ((prof[k][0] / prof[k][1]) * 1e-3) / 1e9) if k in kb and prof[k][1] else None}
               for k in prof}

    adj = None if args.no_adjoint else adjoint_bench(args, dev)
    batch = None if args.no_batch else batch_bench(args, dev)
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
                               "outflow, SSP-RK3 CFL 0.5",
                   "elements": mesh.nel, "K": mesh.K, "dof": dof, "dof_per_var_total": dof * mesh.nvar,
                   "stages_per_step": 3, "blast_center": info["center"]},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "batched": batch,
        "fwd_3d": fwd3d,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
