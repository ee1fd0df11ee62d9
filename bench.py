#!/usr/bin/env python3
"""Throughput benchmark of the entropy-stable DGSEM shallow-water step on one
MI355X.

Workload (default): 512 x 512 curvilinear periodic elements on [0,10]^2
(sin-perturbed map), N = 7 (16.8M LGL nodes), smooth random Fourier state
(h in [0.5,2], |u|,|v| < 0.5, b in [0,1]), full hot path: artificial
viscosity (indicator + BR1), split-form volume term, ES interface flux,
source, LSRK(5,4) stage update with the positivity limiter, adaptive time
step (CFL + viscous + Lemma 2 bounds) computed on the device every step.

Prints ONE JSON line.  value = DOF-updates per second per RK stage
(one DOF = one LGL node with its three unknowns) over the timed steps.
roofline: the fused stage kernel, its algorithmic HBM bytes per launch
divided by its mean launch time (HIP events on the solver stream), against
the 8 TB/s HBM peak.  cpu_baseline: the CPU oracle, one full step and one
right-hand side on a 256 x 256-element patch of the same recipe, with all
host threads and with one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per RK stage (FP64) at N=3..8 + % FP64 roofline; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def geometry_fields(N: int, real_bytes: int) -> int:
    """Geometry the stage kernel reads per node: the four metric directions,
    or, in FP64 at N <= 4, the two coordinates (relative to the element's
    first node) from which it forms them."""
    return 2 if (real_bytes == 8 and N <= 4) else 4


def geometry_elem_fields(real_bytes: int) -> int:
    """Geometry the stage kernel reads per element: in FP32 the four metric
    directions of the element's middle node, to which the stored ones are
    relative."""
    return 4 if real_bytes == 4 else 0


def stage_bytes(N: int, K: int, av: bool, real_bytes: int, stage_index: int, n_visc: int = 0,
                limiter: bool = True) -> float:
    """Algorithmic HBM bytes of one launch of the fused stage kernel: every
    datum the stage must read or write, counted once.
    Reads: W (3/node), dU (3/node, not on the first LSRK stage), metric
    directions (4/node; 2 coordinates at N <= 4 in FP64, geometry_fields;
    in FP32 also 4/element, geometry_elem_fields), split bathymetry
    derivatives (2/node), face
    bathymetry (4(N+1)/element); with AV the element viscosity (1/element)
    and, for the n_visc elements with viscosity, their viscous face fluxes
    (16(N+1)/element, read by their neighbours) and viscous terms (2/node).
    Writes: W (3/node), dU (3/node, not on the last stage: the next step's
    first stage does not read it); on the last stage with the limiter the
    face records of the new state for the next time-step pass (h, u, v at the
    4(N+1) face nodes: 12(N+1)/element)."""
    nf = N + 1
    np_ = nf * nf
    n = K * np_
    per_node = (3 + (3 if stage_index > 0 else 0) + geometry_fields(N, real_bytes) + 2 + 3
                + (3 if stage_index < 4 else 0))
    per_elem = (4 * nf + geometry_elem_fields(real_bytes) + (1 if av else 0)
                + (12 * nf if (limiter and stage_index == 4) else 0))
    visc = (16 * nf + 2 * np_) * n_visc if av else 0
    return (per_node * n + per_elem * K + visc) * real_bytes


def rhs_bytes(N: int, K: int, av: bool, real_bytes: int, n_visc: int = 0) -> float:
    """Algorithmic HBM bytes of one right-hand-side evaluation (the stage
    kernel in its RHS form): reads W (3/node), metric directions (4/node, or
    geometry_fields, and geometry_elem_fields), split bathymetry derivatives (2/node), face bathymetry (4(N+1)/element),
    with AV the element viscosity and the viscous-element terms as in
    stage_bytes; writes R (3/node)."""
    nf = N + 1
    np_ = nf * nf
    visc = (16 * nf + 2 * np_) * n_visc if av else 0
    return ((3 + geometry_fields(N, real_bytes) + 2 + 3) * K * np_
            + (4 * nf + geometry_elem_fields(real_bytes) + (1 if av else 0)) * K + visc) * real_bytes


def av_faces_bytes(N: int, n_visc: int, real_bytes: int) -> float:
    """Algorithmic bytes of the BR1 face-flux pass over n_visc viscous
    elements: per element it reads W (3 (N+1)^2), the neighbours' traces at
    its 4(N+1) face nodes (3 each), the metric directions at its face nodes
    (4 each), its viscosity and face map (4 x (4 + 1) bytes); it writes the
    four viscous flux components at its face nodes (16 (N+1))."""
    nf = N + 1
    return n_visc * ((3 * nf * nf + 12 * nf + 16 * nf + 1 + 16 * nf) * real_bytes + 20)


def av_div_bytes(N: int, n_visc: int, real_bytes: int) -> float:
    """Algorithmic bytes of the viscous-divergence pass: per viscous element
    W (3 (N+1)^2), neighbour traces (12 (N+1)), metric directions
    (4 (N+1)^2), its own and its neighbours' viscosity (5), the neighbours'
    face fluxes (16 (N+1)), the face map; writes L^v (2 (N+1)^2)."""
    nf = N + 1
    np_ = nf * nf
    return n_visc * ((3 * np_ + 12 * nf + 4 * np_ + 5 + 16 * nf + 2 * np_) * real_bytes + 20)


def dt_pass_bytes(N: int, K: int, av: bool, real_bytes: int) -> float:
    """Algorithmic bytes of the time-step pass after a step (the last stage
    left each element's CFL and viscous bounds and its face records): the
    per-element bounds (1 or 2/element), and for the Lemma 2 bounds at every
    face node its record (h, u, v: 3) and the face geometry (unit normal and
    w_0 J/J^surf: 3); the neighbour's record is another element's face node,
    counted there; plus the face map (5 bytes per side)."""
    nf = N + 1
    return K * (((2 if av else 1) + 24 * nf) * real_bytes + 20)


def stage_flops(N: int, av: bool) -> float:
    """Algorithmic FP64 FLOPs per node of one stage (operation count of the
    method, not of this implementation): the volume term 2(N+1) partner pairs
    of 22 FLOP (pairwise sums of the conserved and primitive variables and of
    two metric terms, the contravariant discharge, the two momentum fluxes,
    the D-weighted accumulation), the interface flux (~80 FLOP per face-node
    evaluation, 2(N+1) per element side pair, plus ~36 for the lift, spread
    over the nodes), velocities, source and scaling (~18) and the update
    (~12); with AV the indicator (~20(N+1) + 25); the limiter's test (~15)."""
    nf = N + 1
    f = 44 * nf + 196 / nf + 30 + 15
    if av:
        f += 20 * nf + 25
    return float(f)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_traffic_N7_512x512_fp64.txt")


# the sources that define the stage kernel and its launch
STAGE_SOURCES = ("esdg_inst.hip", "esdg_kernels.hpp", "esdg_launch.hpp", "esdg_tables.hpp")


def kernel_source_hash() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_1804_02221_amd", "csrc")
    h = hashlib.sha256()
    for fn in STAGE_SOURCES:
        h.update(fn.encode())
        with open(os.path.join(src, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per stage-kernel launch from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None when it is missing or was taken on
    other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


ENSEMBLE_GRIDS = (32, 64, 128, 256)
ENSEMBLE_DEGREES = (3, 5, 7)


def ensemble_specs(n_inst: int, seed: int = 4):
    """Batched-ensemble recipe: per instance a grid from {32,...,256}^2, a
    degree from {3, 5, 7}, dam break or bump, its own bathymetry seed."""
    rng = np.random.default_rng(seed)
    return [(int(rng.choice(ENSEMBLE_GRIDS)), int(rng.choice(ENSEMBLE_DEGREES)), bool(rng.integers(2)), seed + i)
            for i in range(n_inst)]


def _member(spec):
    from paper_1804_02221_amd.inputs import ensemble_member
    return ensemble_member(*spec)


def generate_ensemble(specs, workers: int):
    """Generate the members on the host, in worker processes (before any GPU
    use in this process)."""
    if workers <= 1:
        return [_member(sp) for sp in specs]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_member, specs))


def ensemble_bench(esdg, dev, members, steps: int):
    """Time `steps` adaptive steps of all members as one ensemble, then the
    same steps as sequential single-instance solves; DOF-updates per second
    per RK stage over all members."""
    import torch
    nodes = sum(w.mesh.K * (w.mesh.N + 1) ** 2 for w in members)
    ens = esdg.Ensemble(dev, 64)
    for w in members:
        ens.add_workload(w)
    ens.build()
    stages = 3 if members[0].params.get("integrator", 0) == 1 else 5
    ens.step(1, raise_negmean=False)  # warm-up (also builds the time-step bounds)
    tuned = ens.autotune(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_ens = ens.step(steps, raise_negmean=False)
    torch.cuda.synchronize()
    t_ens = time.perf_counter() - t0
    # the same number of further steps with every kernel launched on its own:
    # the difference is the launch overhead the graphs remove
    ens.set_graphs(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(steps, raise_negmean=False)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    ens.close()
    # the same ensemble with the per-instance step check (three retries): a
    # step that met a negative element mean or outran its result's bounds is
    # redone at half the size; one host synchronisation per degree group and step
    ens = esdg.Ensemble(dev, 64)
    for w in members:
        ens.add_workload(w, max_dt_retries=3)
    ens.build()
    ens.step(1, raise_negmean=False)
    ens.autotune(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_retry = ens.step(steps, raise_negmean=False)
    torch.cuda.synchronize()
    t_retry = time.perf_counter() - t0
    ens.close()
    t_seq = 0.0
    negmean_seq = 0
    for w in members:
        s = esdg.solver_for(w, dev)
        s.step(1, 0.0, raise_negmean=False)
        s.autotune(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = s.step(steps, 0.0, raise_negmean=False)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        negmean_seq += int(st != 0)
        s.close()
    return dict(instances=len(members), nodes=nodes, steps=steps, stages_per_step=stages,
                integrator="SSPRK(3,3)" if stages == 3 else "LSRK(5,4)",
                value=nodes * stages * steps / t_ens, ms_per_step=t_ens * 1e3 / steps,
                eager_ms_per_step=t_eager * 1e3 / steps,
                sequential_value=nodes * stages * steps / t_seq, sequential_ms_per_step=t_seq * 1e3 / steps,
                speedup=t_seq / t_ens, stage_variant={str(k): v for k, v in tuned.items()},
                negative_mean_reported={"ensemble": int(st_ens != 0), "sequential_instances": negmean_seq},
                with_step_check={"max_dt_retries": 3, "ms_per_step": t_retry * 1e3 / steps,
                                 "negative_mean_reported": int(st_retry != 0),
                                 "note": "model time differs: redone steps are halved"})


def adjoint_stage_bytes(N: int, K: int) -> float:
    """Algorithmic bytes of one reverse-stage launch, averaged over the five
    stages of a step: per node reads W, dL/dW, the register cotangent (not on a
    step's last stage), the metric directions, b_x, b_y and the three
    bathymetry cotangents; writes dL/dW, the register cotangent (not on the
    first stage) and the three bathymetry cotangents; per element the face
    bathymetry."""
    npn = (N + 1) ** 2
    per_node = (3 + 3 + 0.8 * 3 + 4 + 2 + 3) + (3 + 0.8 * 3 + 3)
    return 8.0 * (K * npn * per_node + K * 4 * (N + 1))


def adjoint_bench(esdg, dev, stream, steps: int = 400, every: int = 20):
    """Bathymetry-gradient workload (128 x 128 elements, N = 5, 32 gauges):
    gauge-misfit loss over `steps` fixed LSRK(5,4) steps against a target run
    over b + db, its gradient by the checkpointed reverse sweep, and the time
    of both against the plain solver's steps."""
    import torch
    from paper_1804_02221_amd.inputs import bathymetry_gradient
    w, x = bathymetry_gradient()
    N = w.mesh.N
    s = esdg.Solver(dev, 64, stream=stream)
    s.upload_mesh(w.mesh)
    s.set_params(esdg.default_params(N, **w.params))
    s.set_bathymetry(w.b)
    s.set_state(w.h, w.hu, w.hv)
    s.set_gauges(x["gelem"], x["gxi"], x["geta"])
    dt = float(s.compute_dt()[0])
    ng = len(x["gelem"])
    zero = np.zeros_like(w.h)
    # target run over b + db
    s.set_bathymetry(w.b + x["db"])
    s.set_state(x["H0"] - w.b - x["db"], zero, zero)
    _, tgt = s.adjoint_forward(steps, dt, every, np.zeros((steps, ng)), want_H=True)
    s.set_bathymetry(w.b)

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # warm-up of every path, then the timed runs
    s.set_state(w.h, w.hu, w.hv)
    s.step(2, dt)
    s.set_state(w.h, w.hu, w.hv)
    s.adjoint_forward(every, dt, every, tgt[:every])
    s.adjoint_backward()
    s.set_state(w.h, w.hu, w.hv)
    _, t_plain = timed(lambda: s.step(steps, dt))
    s.set_state(w.h, w.hu, w.hv)
    loss, t_fwd = timed(lambda: s.adjoint_forward(steps, dt, every, tgt))
    g, t_bwd = timed(lambda: s.adjoint_backward(device=True))
    # the reverse stage kernel alone, timed by events its dispatch records
    s.set_state(w.h, w.hu, w.hv)
    s.adjoint_forward(steps, dt, every, tgt)
    s.profile(True)
    s.profile_read_adjoint()
    s.adjoint_backward(device=True)
    kp = s.profile_read_adjoint()
    s.profile(False)
    K = w.mesh.K
    adj_bytes = adjoint_stage_bytes(N, K)
    adj_mean_ms = kp["ms"] / max(kp["launches"], 1)
    adj_GBs = adj_bytes / (adj_mean_ms * 1e-3) / 1e9
    gb, gh0 = g[0].cpu().numpy(), g[1].cpu().numpy()
    gtot = gb - gh0
    # gradient on the continuous periodic nodes: sum over coincident DG nodes
    lat = np.zeros((w.mesh.nx * N, w.mesh.ny * N))
    np.add.at(lat, (w.mesh.ax, w.mesh.ay), gtot)
    nodes = w.mesh.K * (N + 1) ** 2
    n = nodes * 3 * 8
    s.close()
    return dict(workload=("wet Gaussian surface bump over an 8-Gaussian bed on 128x128 curvilinear periodic "
                          "elements of [0,10]^2, N=5, AV off, limiter on (inactive), ES flux, 32 gauges, "
                          "target run over b + db"),
                nodes=nodes, steps=steps, checkpoint_every=every, gauges=ng, dt=dt, loss=loss,
                plain_forward_ms=t_plain * 1e3, forward_ms=t_fwd * 1e3, backward_ms=t_bwd * 1e3,
                adjoint_forward_ratio=t_bwd / t_plain, total_ratio=(t_fwd + t_bwd) / t_plain,
                backward_value=nodes * 5 * steps / t_bwd,
                gradient_values=int(gtot.size), continuous_nodes=int(lat.size),
                gradient_norm=float(np.linalg.norm(gtot)), continuous_gradient_norm=float(np.linalg.norm(lat)),
                checkpoint_bytes=((steps + every - 1) // every) * n, segment_bytes=(every * 5 + 1) * n,
                roofline={"bound": "hbm", "kernel": "adjoint_stage_kernel", "achieved": adj_GBs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": adj_GBs / HBM_PEAK_GBS,
                          "bytes_per_launch": adj_bytes, "mean_launch_ms": adj_mean_ms,
                          "launches": kp["launches"], "traffic": None})


def paper_cases_bench(esdg, dev, stream):
    """The paper's walled test cases at their own resolutions, SSPRK(3,3) with
    the adaptive step: the oscillating lake (200x200, N=3) to T/6 with its
    error against the closed form, the dry dam break (50x50, N=3) to t=1 and
    the dam break over three mounds (150x100, N=3) to t=10 (~25000 steps;
    the paper shows it up to t=50) and the run-up on a conical island
    (50x50, N=3) to t=50, with their mass drift and entropy change."""
    import torch
    from paper_1804_02221_amd.inputs import conical_island, dry_dam_break, oscillating_lake, three_mound_dam_break
    out = {}
    g = 9.81
    for name, w, t_end in (("oscillating_lake", oscillating_lake(200, 3), 2 * np.pi / np.sqrt(2 * g * 0.1) / 6),
                           ("dry_dam_break", dry_dam_break(50, 3), 1.0),
                           ("three_mound_dam_break", three_mound_dam_break(150, 100, 3), 10.0),
                           ("conical_island", conical_island(50, 50, 3), 50.0)):
        s = esdg.Solver(dev, 64, stream=stream)
        s.upload_mesh(w.mesh)
        s.set_params(esdg.default_params(3, **w.params))
        s.set_bathymetry(w.b)
        s.set_state(w.h, w.hu, w.hv)
        d0 = s.diagnostics()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, n = 0.0, 0
        while t < t_end - 1e-12:
            dt = min(s.compute_dt()[0], t_end - t)
            t, _ = s.step(1, dt)
            n += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = s.diagnostics()
        nodes = w.mesh.K * 16
        r = dict(elements=w.mesh.K, nodes=nodes, t_end=t_end, steps=n, ms_per_step=el * 1e3 / n,
                 value=nodes * 3 * n / el, mass_drift=(d[0] - d0[0]) / d0[0], entropy_change=(d[3] - d0[3]) / d0[3],
                 min_h=d[5])
        if name == "oscillating_lake":
            h = s.get_state()[0]
            ex = oscillating_lake(200, 3, t=t_end)
            geo = s.get_geometry()
            w1 = np.array([1 / 6, 5 / 6, 5 / 6, 1 / 6])   # LGL weights, N = 3
            wq = geo["J"] * np.outer(w1, w1).reshape(-1)[None, :]
            r["relative_L1_error"] = float(np.sum(wq * np.abs(h - ex.h)) / np.sum(wq * ex.h))
        r["viscous_elements_at_end"] = int((s.get_eps() > 0).sum())
        s.close()
        out[name] = r
    out["note"] = ("wall-clock per step includes the host loop (one esdg_step and one esdg_compute_dt per step, "
                   "the step clipped to reach t_end); value = nodes x 3 stages x steps / elapsed")
    return out


def host_threads() -> int:
    """Host threads the oracle may use: the CPU share this process has (the
    OpenMP setting when given, else the CPUs it may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N: int, n_patch: int):
    """The CPU oracle (test infrastructure, never tuned) on a bounded sample
    of the timed workload: one full LSRK(5,4) step and one right-hand side on
    an n_patch^2-element patch of the same recipe, with all the host threads
    it has and with one."""
    import oracle
    from paper_1804_02221_amd.inputs import smooth_sweep
    w = smooth_sweep(n_patch, N, seed=3)
    P = oracle.params(N, av_on=1, limiter_on=1, eps0=0.025)
    nodes = w.mesh.K * (N + 1) ** 2
    threads = host_threads()
    out = {}
    for label, nt in (("all", threads), ("one", 1)):
        oracle.set_threads(nt)
        t0 = time.perf_counter()
        oracle.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0)
        t_step = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
        t_rhs = time.perf_counter() - t0
        out[label] = (t_step, t_rhs)
        log(f"CPU oracle, {nt} thread(s): step {t_step:.2f} s, rhs {t_rhs:.2f} s")
    oracle.set_threads(threads)
    t_step, t_rhs = out["all"]
    return dict(value=nodes * 5 / t_step, unit="DOF-updates/s", cores=threads, kind="oracle",
                sample=(f"one LSRK(5,4) step (5 stages, AV + limiter + adaptive dt) on a {n_patch}x{n_patch}-"
                        f"element patch of the same recipe, N={N} ({nodes} nodes), {threads} OpenMP threads "
                        f"over elements, {t_step:.2f} s"),
                cpu_model=cpu_model(),
                rhs_only={"value": nodes / t_rhs, "unit": "DOF/s (one right-hand side)", "seconds": t_rhs},
                single_thread={"value": nodes * 5 / out["one"][0], "step_seconds": out["one"][0],
                               "rhs_value": nodes / out["one"][1], "rhs_seconds": out["one"][1], "cores": 1})


def kernel_times(prof, steps: int):
    """ms per step of each timed kernel class (profile_read_kernels)."""
    return {k: {"ms_per_step": ms / steps, "launches": n, "mean_launch_ms": ms / n if n else 0.0}
            for k, (ms, n) in prof.items() if n}


def dam_break_bench(esdg, dev, stream, steps: int, warmup: int):
    """The curvilinear wet/dry dam break (128x128 elements, N=7, AV with
    eps0=0.025, limiter, LSRK(5,4), adaptive step): the hot path with its
    non-smooth parts active.  Reports the stage kernel (bytes including the
    viscous elements' terms), the two viscosity passes and the time-step
    pass against the HBM peak, the viscous and limited counts."""
    import torch
    from paper_1804_02221_amd.inputs import dam_break
    w = dam_break(128, 7)
    N, K = 7, w.mesh.K
    nodes = K * (N + 1) ** 2
    s = esdg.Solver(dev, 64, stream=stream)
    s.upload_mesh(w.mesh)
    s.set_params(esdg.default_params(N, **w.params))
    s.set_bathymetry(w.b)
    s.set_state(w.h, w.hu, w.hv)
    s.step(warmup, 0.0, raise_negmean=False)
    _, v0 = s.step_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_sim, st_run = s.step(steps, 0.0, raise_negmean=False)     # graph replay
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    limited, v1 = s.step_stats()
    # the next steps of the run, every kernel on its own with timing events
    s.profile(True)
    s.profile_read_kernels()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st2 = s.step(steps, 0.0, raise_negmean=False)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    prof = s.profile_read_kernels()
    s.profile(False)
    st_run = st_run or st2
    d = s.diagnostics()
    s.close()
    n_visc = 0.5 * (v0 + v1)
    st_ms, st_n = prof["stage"]
    stage_b = sum(stage_bytes(N, K, True, 8, k, int(round(n_visc))) for k in range(5)) / 5
    res = dict(workload=("curvilinear wet/dry dam break, 128x128 elements of [0,10]^2, N=7, 8-Gaussian bottom, "
                         "AV eps0=0.025 + limiter, ES flux, LSRK(5,4), adaptive dt (CFL, viscous, Lemma 2)"),
               nodes=nodes, steps=steps, warmup=warmup, t_sim=t_sim, min_h=d[5],
               value=nodes * 5 * steps / el, unit="DOF-updates/s", ms_per_step=el * 1e3 / steps,
               eager_ms_per_step=el_eager * 1e3 / steps,
               viscous_elements={"before": v0, "after": v1}, limited_element_stages=limited,
               negative_mean_reported=int(st_run != 0),
               kernels=kernel_times(prof, steps))
    rl = {}
    if st_n:
        t = st_ms / st_n * 1e-3
        rl["stage_kernel"] = {"bytes_per_launch": stage_b, "GBs": stage_b / t / 1e9,
                              "frac": stage_b / t / 1e9 / HBM_PEAK_GBS}
    for k, fn in (("av_faces", av_faces_bytes), ("av_div", av_div_bytes)):
        ms, n = prof[k]
        if n:
            b = fn(N, n_visc, 8)
            rl[k + "_kernel"] = {"bytes_per_launch": b, "GBs": b / (ms / n * 1e-3) / 1e9,
                                 "frac": b / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "note": "bytes of the listed viscous elements only (mean count)"}
    ms, n = prof["dt"]
    if n:
        b = dt_pass_bytes(N, K, True, 8)
        rl["dt_pass"] = {"bytes_per_launch": b, "GBs": b / (ms / n * 1e-3) / 1e9,
                         "frac": b / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS}
    res["roofline"] = rl
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=7)
    ap.add_argument("--n", type=int, default=512, help="elements per side")
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32))
    ap.add_argument("--no-av", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-patch", type=int, default=256)
    ap.add_argument("--sweep", default="2,3,4,5,6,8",
                    help="comma list of further N values to time on the same mesh ('' for none)")
    ap.add_argument("--sweep-steps", type=int, default=10)
    ap.add_argument("--fp32-sweep", type=int, default=1,
                    help="also time FP32 at the main N and every sweep N, with its error against FP64")
    ap.add_argument("--rhs-reps", type=int, default=10, help="right-hand-side evaluations timed per N")
    ap.add_argument("--dam-break", type=int, default=1,
                    help="time the 128^2 N=7 wet/dry dam break (AV and limiter active)")
    ap.add_argument("--dam-break-steps", type=int, default=100)
    ap.add_argument("--ensemble", type=int, default=64,
                    help="instances of the batched-ensemble comparison (0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--adjoint", type=int, default=1,
                    help="time the bathymetry-gradient adjoint (128^2 elements, N=5, 400 steps)")
    ap.add_argument("--paper-cases", type=int, default=0,
                    help="run the walled test cases (oscillating lake, dry dam break) at their resolutions")
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick the stage-kernel tile per run with the library's autotuner")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(the halo exchange over several GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    members = []
    if args.ensemble > 0:
        log(f"generating the {args.ensemble}-instance ensemble on the host")
        t0 = time.perf_counter()
        members = generate_ensemble(ensemble_specs(args.ensemble), min(16, host_threads()))
        log(f"ensemble generated in {time.perf_counter() - t0:.1f} s")

    import torch
    from paper_1804_02221_amd import esdg
    from paper_1804_02221_amd.inputs import smooth_sweep

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream()

    def run(w, N, precision, steps, warmup, rhs_reps, fp64_rhs=None):
        s = esdg.Solver(dev, precision, stream=stream)
        s.upload_mesh(w.mesh)
        P = esdg.default_params(N, av_on=0 if args.no_av else 1, limiter_on=1, eps0=0.025)
        s.set_params(P)
        s.set_bathymetry(w.b)
        s.set_state(w.h, w.hu, w.hv)
        K = w.mesh.K
        nodes = K * (N + 1) ** 2
        av = not args.no_av
        rb = 8 if precision == 64 else 4
        # right-hand side alone: the stage kernel in its RHS form, events per launch
        s.rhs(device=True)
        s.profile(True)
        s.profile_read_kernels()
        for _ in range(rhs_reps):
            R = s.rhs(device=True)
        prof = s.profile_read_kernels()
        s.profile(False)
        rhs_ms = prof["stage"][0] / max(prof["stage"][1], 1)
        rhs_b = rhs_bytes(N, K, av, rb)
        err32 = None
        rel = lambda x, y: [float((a - b).abs().max() / b.abs().max()) for a, b in zip(x, y)]
        if fp64_rhs is not None:
            R64, R64r = fp64_rhs
            err32 = {"max_abs_over_max": rel(R, R64),
                     "l2_relative": [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                                     for a, b in zip(R, R64)],
                     # the FP64 path on the state rounded to FP32: the part of the error that
                     # storing the state in FP32 costs, whatever the arithmetic (both paths take
                     # the bathymetry in FP64; FP32 rounds only its derivatives and face values)
                     "input_rounding_floor": rel(R64r, R64),
                     # against that: the FP32 arithmetic and the FP32 metric terms
                     "vs_fp64_on_rounded_inputs": rel(R, R64r),
                     "fields": ["h", "hu", "hv"], "state": "initial state of the workload"}
            log(f"N={N} FP32 rhs vs FP64: max-abs / max {max(err32['max_abs_over_max']):.2e}; "
                f"input rounding alone {max(err32['input_rounding_floor']):.2e}; "
                f"vs FP64 on the rounded inputs {max(err32['vs_fp64_on_rounded_inputs']):.2e}")
            R = None
        elif precision == 64:
            R = [r.clone() for r in R]
            f32 = lambda x: x.astype(np.float32).astype(np.float64)
            s.set_state(f32(w.h), f32(w.hu), f32(w.hv))
            R = (R, [r.clone() for r in s.rhs(device=True)])
            s.set_state(w.h, w.hu, w.hv)
        else:
            R = None
        s.step(warmup, 0.0)
        choice, tune_ms = s.autotune(20) if args.autotune else (0, None)
        s.step(3, 0.0)        # one step from each state buffer: the step graphs are captured here
        torch.cuda.synchronize()
        # the timed steps: each step one graph replay (esdg_set_graphs)
        t0 = time.perf_counter()
        t_sim, _ = s.step(steps, 0.0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # the same number of steps again, every kernel launched on its own with
        # timing events (per-kernel figures; eager step time for comparison)
        s.profile(True)
        s.profile_read_kernels()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, 0.0)
        torch.cuda.synchronize()
        el_eager = time.perf_counter() - t0
        prof = s.profile_read_kernels()
        s.profile(False)
        limited, n_visc = s.step_stats()
        d = s.diagnostics()
        log(f"N={N} FP{precision}: {steps} steps in {el:.3f} s, t={t_sim:.4g}, min h={d[5]:.3g}, "
            f"stage variant {choice}")
        per_step = sum(stage_bytes(N, K, av, rb, k, n_visc) for k in range(5))
        st_ms, st_n = prof["stage"]
        stage_mean_ms = st_ms / max(st_n, 1)
        achieved = per_step * steps / (st_ms * 1e-3) / 1e9
        flops_node = stage_flops(N, av)
        kt = kernel_times(prof, steps)
        outside = sum(v["ms_per_step"] for k, v in kt.items() if k != "stage")
        res = dict(N=N, precision=precision, K=K, nodes=nodes, elapsed=el, t_sim=t_sim, n_visc=n_visc,
                   limited_element_stages=limited,
                   stage_TFLOPs=flops_node * nodes / (stage_mean_ms * 1e-3) / 1e12,
                   flops_per_node=flops_node, stage_variant=choice,
                   autotune_ms=list(tune_ms) if tune_ms is not None else None,
                   value=nodes * 5 * steps / el, ms_per_step=el * 1e3 / steps,
                   eager_ms_per_step=el_eager * 1e3 / steps,
                   stage_mean_ms=stage_mean_ms, stage_launches=st_n,
                   stage_bytes_per_launch=per_step / 5, stage_GBs=achieved,
                   roofline_frac=achieved / HBM_PEAK_GBS,
                   kernels_ms_per_step=kt, outside_stage_ms_per_step=outside,
                   rhs_only={"kernel_ms": rhs_ms, "value": nodes / (rhs_ms * 1e-3), "unit": "DOF/s (one RHS)",
                             "bytes": rhs_b, "GBs": rhs_b / (rhs_ms * 1e-3) / 1e9,
                             "frac": rhs_b / (rhs_ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
        if err32 is not None:
            res["fp32_vs_fp64_rhs"] = err32
        s.close()
        return res, R

    keys = ("N", "precision", "nodes", "value", "ms_per_step", "eager_ms_per_step", "stage_mean_ms", "stage_GBs",
            "roofline_frac",
            "stage_TFLOPs", "stage_variant", "autotune_ms", "outside_stage_ms_per_step", "rhs_only")
    sweep = []
    main_res = None
    degrees = [args.N] + [int(t) for t in args.sweep.split(",") if t.strip() and int(t) != args.N]
    for N in degrees:
        log(f"generating {args.n}x{args.n} workload at N={N}")
        w = smooth_sweep(args.n, N, seed=3)
        is_main = N == args.N
        steps = args.steps if is_main else args.sweep_steps
        warm = args.warmup if is_main else 2
        r64, R64 = run(w, N, args.precision, steps, warm, args.rhs_reps)
        if is_main:
            main_res = r64
        else:
            sweep.append({k: r64[k] for k in keys})
        if args.fp32_sweep and args.precision == 64:
            r32, _ = run(w, N, 32, args.sweep_steps, 2, args.rhs_reps, fp64_rhs=R64)
            sweep.append({k: r32[k] for k in keys + ("fp32_vs_fp64_rhs",) if k in r32})
        del w, R64
        torch.cuda.empty_cache()

    log("memcopy probe")
    mc = memcopy_probe(torch, dev, main_res["stage_bytes_per_launch"])
    log("LDS probe")
    lds_bw = esdg.lds_bandwidth(dev)
    # LDS bytes the volume term reads per node: 2(N+1) partners x (metric pair, discharge
    # pair, velocity pair: 16 B each; h and the D entry: 8 B each)
    lds_node = 2 * (args.N + 1) * 64.0
    lds_achieved = lds_node * main_res["nodes"] / (main_res["stage_mean_ms"] * 1e-3)

    dam = None
    if args.dam_break:
        log("128^2 N=7 wet/dry dam break")
        dam = dam_break_bench(esdg, dev, stream, args.dam_break_steps, 5)

    ens = None
    if members:
        log("ensemble vs sequential solves")
        ens = ensemble_bench(esdg, dev, members, args.ensemble_steps)
        ens["recipe"] = ("grids {32,64,128,256}^2, N in {3,5,7}, dam break or Gaussian bump over a "
                         "Gaussian-sum bed, AV + limiter, SSPRK(3,3) (the paper's wet/dry integrator), "
                         "adaptive dt per instance")
        del members

    adj = None
    if args.adjoint:
        log("bathymetry-gradient adjoint")
        adj = adjoint_bench(esdg, dev, stream)
        log(f"adjoint: backward / plain forward = {adj['adjoint_forward_ratio']:.2f}")

    cases = None
    if args.paper_cases:
        log("walled test cases")
        cases = paper_cases_bench(esdg, dev, stream)

    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        log(f"CPU oracle baseline on a {args.cpu_patch}^2 patch")
        cpu = cpu_baseline(args.N, args.cpu_patch)

    frac = main_res["stage_GBs"] / HBM_PEAK_GBS
    traffic = None
    if args.N == 7 and args.n == 512 and args.precision == 64 and not args.no_av:
        traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "eager_ms_per_step": main_res["eager_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"smooth random Fourier state on {args.n}x{args.n} curvilinear periodic "
                         f"elements of [0,10]^2, N={args.N}, {'AV + ' if not args.no_av else ''}"
                         f"limiter, ES flux, LSRK(5,4), adaptive dt"),
            "N": args.N, "elements": main_res["K"], "nodes": main_res["nodes"],
            "stage_variant": main_res["stage_variant"],
            "autotune_ms": main_res["autotune_ms"],
            "stages_per_step": 5, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": main_res["stage_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": frac, "traffic": traffic, "kernel": "stage_kernel",
            "bytes_per_launch": main_res["stage_bytes_per_launch"],
            "viscous_elements": main_res["n_visc"],
            "mean_launch_ms": main_res["stage_mean_ms"],
            f"fp{args.precision}_vector": {"achieved_TFLOPs": main_res["stage_TFLOPs"],
                            "peak_TFLOPs": 78.6 if args.precision == 64 else 157.3,
                            "flops_per_node": main_res["flops_per_node"],
                            "note": "algorithmic FLOPs of the method (bench.stage_flops)"},
        },
        "cpu_baseline": cpu,
        "kernels_ms_per_step": main_res["kernels_ms_per_step"],
        "outside_stage_ms_per_step": main_res["outside_stage_ms_per_step"],
        "rhs_only": main_res["rhs_only"],
        "memcopy_roofline": {"GBs": mc["GBs"], "bytes": mc["bytes"],
                             "stage_frac": main_res["stage_GBs"] / mc["GBs"]},
        "lds_roofline": {"probe_GBs": lds_bw / 1e9, "volume_bytes_per_node": lds_node,
                         "stage_volume_GBs": lds_achieved / 1e9, "frac": lds_achieved / lds_bw},
    }
    if sweep:
        out["sweep"] = sweep
    if dam:
        out["dam_break"] = dam
    if ens:
        out["ensemble"] = ens
    if adj:
        out["adjoint"] = adj
    if cases:
        out["paper_cases"] = cases
    print(json.dumps(out), flush=True)


def memcopy_probe(torch, dev, nbytes):
    """The paper's empirical MemCopy roofline: a device copy moving the
    stage's bytes ((read + written)/2 each way), timed with events."""
    n = int(nbytes // 2 // 8)
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return dict(bytes=2 * n * 8, mean_ms=ms, GBs=2 * n * 8 / (ms * 1e-3) / 1e9)


if __name__ == "__main__":
    main()
