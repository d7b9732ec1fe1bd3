#!/usr/bin/env python3
"""Benchmark of the sub-grid DG shallow-water step on one MI355X.

Metric: FP64 DoF-updates per second per RK stage (stored nodal values of
zeta, qx, qy (and c with a tracer) times the stages taken, over the timed
wall time), on the 256x256, r = 2, 16x16-sample beach dam break (SSP3), with
every input resident in device memory before the timed region.

One JSON line is printed.  `value` comes from a timed region with no
per-kernel events.  Besides the metric the line carries
  roofline:     the dominant kernel's algorithmic bytes and flops per launch
                divided by its average launch time, from HIP events the
                library records (on its stream, fence-free) around that
                kernel's launches only, in a second timed pass over the same
                steps from the same start; kernel_share comes from a third
                pass with every kernel class timed;
  quadtree:     the 2-level quadtree with tracer, tide and hanging faces
                (about 120k leaves, r = 3): DoF-updates/s of its coupled step;
  ensemble:     ensemble_64, batched + graph-replayed vs one by one;
  adjoint:      adjoint_128 gradient, backward vs forward time;
  imex:         the same beach case stepped with the IMEX pair (friction by
                the TR-BDF2 companion) and with plain RK32, DoF-updates/s;
  vortex:       the travelling vortex of Sec. 4.4 on the paper's finest static
                mesh (640 x 320 cells) to T = 1/6 s with each scheme of its
                table (RK32 r = 1, SSP3 r = 2, RK44 r = 3): wall time next to
                the paper's CPU wall time for the same run (8 processes);
  cpu_baseline: the oracle timed on the host cores on a bounded window of
                the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (and matrix) peak
# VALU issue: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every 4
# cycles at 2.4 GHz (FP64 FMA: 16 lanes x 2 flops x 4 SIMDs x 256 CUs x 2.4 GHz
# = 78.6 TFLOP/s)
N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9
VALU_CYCLES = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "element_stage_beach_dambreak_256.traffic.json")
STAGE_SOURCES = ["sw_stage.inc", "sw_dev.h", "sw_internal.h", "sw_stage_dispatch.inc", "sw_stage_r2.hip"]
# the fast tracer kernel also inlines the element kernels' helpers
TRACER_SOURCES = STAGE_SOURCES + ["sw_tracer.inc", "sw_tracer_r3.hip"]


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2505_18743_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stage_source_sha():
    return source_sha(STAGE_SOURCES)


def tracer_source_sha():
    return source_sha(TRACER_SOURCES)


def element_stage_work(S, r, n_f, stage_terms):
    """Algorithmic bytes and flops per cell of one launch of the fast element
    kernel of a stage (Newton first iterate, discharge update, one pass over
    the samples that verifies the iterate and integrates the volume terms):

    bytes = 8 [ S^2                      bathymetry samples
              + 3 NP                     zeta^n, q^n
              + 2 NP                     H(zeta^n), all-wet B
              + n_f NP m                 m stored stage residuals read
              + n_f NP                   volume residual written
              + n_f NP ]                 stage state written
    flops = S^2 [ 2 (r+1) 5              interpolation of zeta, d_x zeta, d_y zeta, qx, qy
              + 2 (r+1) 8               8 test-function accumulations (F: 2, Gx: 3, Gy: 3)
              + 40 ]                     pointwise h, 1/h_des, u, friction, sources, fluxes
            + 2 NP^2 n_f                M0^{-1} (zeta) and exact-mass inverse (qx, qy)
    with NP = (r+1)^2 and m the number of stored residuals combined.
    """
    NP = (r + 1) ** 2
    words = S * S + 5 * NP + n_f * NP * (stage_terms + 2)
    flops = S * S * (2 * (r + 1) * 5 + 2 * (r + 1) * 8 + 40) + 2 * NP * NP * n_f
    return 8.0 * words, float(flops)


def tracer_stage_work(S, r, stage_terms):
    """Algorithmic bytes and flops per cell of one launch of the fast tracer
    kernel of a stage (tracer target, h-weighted matrix from one pass over
    the samples, Cholesky solve, tracer volume residual of the new state):

    bytes = 8 [ S^2                      bathymetry samples
              + 3 NP                     zeta, qx, qy of the stage
              + 2 NP                     c^n, C~^n
              + NP m                     m stored tracer residuals
              + 2 NP ]                   new c and its residual written
    flops = S^2 [ 2 (r+1)                zeta at the node
              + 2 NX                     x-pair partials of int h psi_i psi_j
              + 2 (r+1) 3                qx, qy, c at the node
              + 2 (r+1) 2 ]              residual accumulations
            + 2 S NT + NP^3 / 3 + 2 NP^2 assembly along y, factorisation, solves
    with NP = (r+1)^2, NX = (r+1)(r+2)/2, NT = NP (NP+1)/2.
    """
    NP = (r + 1) ** 2
    NX = (r + 1) * (r + 2) // 2
    NT = NP * (NP + 1) // 2
    words = S * S + NP * (7 + stage_terms)
    flops = S * S * (2 * (r + 1) + 2 * NX + 6 * (r + 1) + 4 * (r + 1)) + 2 * S * NT + NP ** 3 / 3 + 2 * NP * NP
    return 8.0 * words, float(flops)


def lanes_for(S):
    """Lanes per cell of the element kernels: the power of two >= S (at least 4)."""
    P = 4
    while P < S:
        P <<= 1
    return P


def read_counters(path, sha):
    """A counter record of profiles/ taken on the current kernel sources (else None)."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    return tr if tr.get("source_sha") == sha else None


def roofline(bytes_launch, flops_launch, launch_s, counters, kernel):
    """Roofline of one kernel launch.  achieved = algorithmic bytes (flops) per
    launch / launch time.  The bound is the resource the counters show busier:
    HBM (counter bytes / launch time against the 8 TB/s peak) or VALU issue
    (VALU instructions x 4 cycles against 1,024 SIMDs at 2.4 GHz); an
    issue-bound kernel reports its FP64 rate against the FP64 peak ("alu").
    Without a counter record for the current sources the larger of the two
    algorithmic fractions decides."""
    gbs = bytes_launch / launch_s / 1e9
    tfl = flops_launch / launch_s / 1e12
    f_hbm, f_fp = gbs / HBM_PEAK_GBS, tfl / FP64_PEAK_TFLOPS
    traffic = issue = hbm_counter = None
    if counters:
        traffic = counters.get("bytes_per_launch")
        if traffic:
            hbm_counter = traffic / launch_s / 1e9 / HBM_PEAK_GBS
        vi = counters.get("valu_insts_per_launch")
        if vi:
            issue = vi * VALU_CYCLES / (N_SIMD * CLOCK_HZ * launch_s)
    if issue is not None and hbm_counter is not None:
        alu = issue > hbm_counter
        basis = "counters"
    else:
        alu = f_fp > f_hbm
        basis = "algorithmic fractions (no counter record for these sources)"
    if alu:
        roof = dict(bound="alu", achieved=round(tfl, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=round(f_fp, 4))
    else:
        roof = dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(f_hbm, 4))
    roof.update(traffic=traffic, kernel=kernel, launch_ms=round(launch_s * 1e3, 5),
                algo_bytes_per_launch=bytes_launch, algo_flops_per_launch=flops_launch,
                hbm_frac=round(f_hbm, 4), fp64_frac=round(f_fp, 4), bound_from=basis,
                valu_issue_frac=None if issue is None else round(issue, 4),
                hbm_frac_counters=None if hbm_counter is None else round(hbm_counter, 4))
    return roof


_T0 = time.perf_counter()


def progress(what):
    """One line on stderr as each part of the run starts (stdout keeps the JSON line)."""
    print(f"bench: {time.perf_counter() - _T0:7.1f} s  {what}", file=sys.stderr, flush=True)


def copy_roof(device, mib=1024, reps=10):
    """Attainable HBM bandwidth on this GPU: a device-to-device copy of `mib`
    MiB (read plus write) through the runtime's copy kernel, event-timed."""
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device=device)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n / (ms * 1e-3) / 1e9


def calibration_copy(mib, device):
    """Two device-to-device copies of `mib` MiB: a kernel of known traffic for
    scaling the HBM counters of a profiled run."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=device)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def setup(wl, device):
    import numpy as np
    from paper_2505_18743_amd import Solver
    s = Solver(wl["mesh"], wl["params"], device=device)
    xy = s.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    s.set_bathymetry(b)
    s.set_manning(wl["manning"])
    dof = s.dof_coords()
    eta0 = wl["eta0"](dof[:, 0], dof[:, 1])
    c0 = wl["tracer0"](dof[:, 0], dof[:, 1]) if wl.get("tracer0") else None

    def reset():
        s.init_lake_at_rest(eta0)
        st = s.get_state()
        s.set_state(st[0], st[1], st[2], c0 if c0 is not None else None)
        s.set_time(0.0)
    reset()
    return s, reset, np.asarray(b)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, window=(96, 96, 64, 64)):
    """The oracle (PyTorch CPU, float64) on the host: one SSP3 step of the
    whole mesh after one warm-up step with every host thread torch uses, and
    one step of a 64x64 window of it after a warm-up step on one thread."""
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import build_oracle
    from workloads import workload
    from oracle import tableau

    def rate(wl, threads):
        torch.set_num_threads(threads)
        o, _ = build_oracle(wl)
        stages = len(tableau(o.p.rk)[1])
        dofs = (3 + (1 if o.p.tracer else 0)) * o.np_ * o.m.K
        o.step()                      # warm-up
        t0 = time.perf_counter()
        o.step()
        el = time.perf_counter() - t0
        return dofs * stages / el, el, o.m.K

    threads = torch.get_num_threads()
    full, el_full, K_full = rate(workload(name), threads)
    progress("cpu baseline: one thread")
    one, el_one, K_one = rate(workload(name, window=window) if name == "beach_dambreak_256" else workload(name), 1)
    torch.set_num_threads(threads)
    return dict(value=full, unit="DoF-updates/s", cores=threads, kind="oracle",
                sample=f"oracle on the whole {name} mesh ({K_full} cells), 1 SSP3 step after 1 warm-up step, "
                       f"{el_full:.1f} s, {threads} threads",
                nproc=os.cpu_count(), cpu_model=cpu_model(),
                one_core=dict(value=one, unit="DoF-updates/s", cores=1,
                              sample=f"oracle on a {K_one}-cell window (64x64) of {name}, 1 SSP3 step after 1 "
                                     f"warm-up step, {el_one:.1f} s, 1 thread"))


def quadtree_bench(steps, warmup, device):
    """The 2-level quadtree with about 120k leaves (r=3, 32/16/8 samples per
    level, tracer, tide, hanging faces): DoF-updates/s of the coupled step
    (zeta, qx, qy and the tracer), and the kernel classes' shares."""
    import torch
    from workloads import workload
    wl = workload("tidal_quadtree_r3")
    s, reset, _ = setup(wl, device)
    stages = {"fe": 1, "ssp3": 3, "rk32": 3, "rk44": 4}[wl["params"]["rk"]]
    dofs_stage = 4 * (int(wl["params"]["r"]) + 1) ** 2 * s.n_cells
    s.run(warmup)
    s.sync()
    reset()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    s.run(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    diag = s.diagnostics()
    reset()
    torch.cuda.synchronize()
    s.profile(True)
    s.kernel_time_reset()
    ev0.record()
    s.run(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms2 = ev0.elapsed_time(ev1)
    kt = s.kernel_times()
    s.profile(False)
    s.close()
    # roofline of the heavier of the stage-mode element and tracer kernels:
    # their launches over the timed steps (one per level and stage) against
    # the algorithmic bytes and flops of every cell of every level
    r = int(wl["params"]["r"])
    Ss = wl["params"]["S"]
    lev = wl["mesh"]["level"]
    per_level = [int((lev == L).sum()) for L in range(len(Ss))]
    mean_terms = sum(range(1, stages)) / max(stages - 1, 1)
    calls = steps * (stages - 1)
    cand = {}
    for name, work in (("element_stage", lambda S: element_stage_work(S, r, 3, mean_terms)),
                       ("element_tracer", lambda S: tracer_stage_work(S, r, mean_terms))):
        t_ms, n = kt[name]
        if n == 0:
            continue
        b = sum(k * work(S)[0] for k, S in zip(per_level, Ss)) * calls
        f = sum(k * work(S)[1] for k, S in zip(per_level, Ss)) * calls
        cand[name] = (t_ms, b, f, n)
    roof = None
    if cand:
        name = max(cand, key=lambda k: cand[k][0])
        t_ms, b, f, n = cand[name]
        kname = "k_elem" if name == "element_stage" else "k_trc"
        kernel = f"{kname}<r={r},P={'/'.join(str(lanes_for(S)) for S in Ss)},F_STAGE> (one launch per level)"
        counters = read_counters(os.path.join(ROOT, "profiles", f"{name}_tidal_quadtree_r3.traffic.json"),
                                 stage_source_sha() if name == "element_stage" else tracer_source_sha())
        # per stage: the launches of all levels together
        roof = roofline(b / calls, f / calls, t_ms * 1e-3 / calls, counters, kernel)
        roof.update(launches=n, scope="all levels of one stage per launch group")
    return dict(workload="tidal_quadtree_r3", cells=s.n_cells, steps=steps, ms_per_step=ms / steps,
                value=dofs_stage * stages * steps / (ms * 1e-3), unit="DoF-updates/s",
                fields=4, r0_cells=diag["n_r0_cells"], max_newton_it=diag["max_newton_it"],
                kernel_share={k: round(v[0] / ms2, 4) for k, v in kt.items()}, roofline=roof)


def ensemble_bench(steps, warmup, device, eager_only=False):
    """64-member ensemble (uneven meshes, r in {1,2,3}): batched and graph-
    replayed vs the same members as 64 contexts stepped one after another.
    eager_only: just `steps` eager batched steps with the default launch
    shapes (for a profiler)."""
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import member_solver, setup_ensemble
    from workloads import workload
    mem = workload("ensemble_64")
    ens, inputs = setup_ensemble(mem, device)
    if eager_only:
        ens.run(steps, graph=False)
        ens.sync()
        ens.close()
        return dict(workload="ensemble_64", members=len(mem), steps=steps, mode="eager, default launch shapes")
    tuned = ens.autotune(steps=3)      # launch shape per degree class (state restored)
    stages = 3
    dofs = sum(3 * (w["params"]["r"] + 1) ** 2 * len(w["mesh"]["level"]) for w in mem)
    cells = sum(len(w["mesh"]["level"]) for w in mem)

    def reset_ens():
        for s, (bed, man, eta) in zip(ens.batches, inputs):
            s.init_lake_at_rest(eta)
            s.set_time(0.0)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    res = {}
    for mode, graph in (("graph", True), ("eager", False)):
        reset_ens()
        ens.run(warmup, graph=graph)
        ens.sync()
        reset_ens()
        ens.run(1, graph=graph)   # the first step after a reset is taken eagerly
        ens.sync()
        res[mode] = timed(lambda: ens.run(steps, graph=graph))
        ens.sync()
    ones = [member_solver(ens, inputs, mem, m, device) for m in range(len(mem))]
    for m, o in enumerate(ones):         # the same launch shapes one by one
        t = tuned[ens.where[m][0]]
        o.set_workgroup(t["elem_waves_per_workgroup"], kernel=0)
        o.set_workgroup(t["face_lanes"], kernel=1)
    etas = []
    for m in range(len(mem)):
        b, i = ens.where[m]
        etas.append(inputs[b][2][ens.batches[b].member_index(i)[2]])
    for o in ones:
        o.run(warmup)
    for o, eta in zip(ones, etas):
        o.init_lake_at_rest(eta)
        o.set_time(0.0)
        o.run(1)

    def one_by_one():
        for o in ones:
            o.run(steps)
    res["one_by_one"] = timed(one_by_one)
    for o in ones:
        o.close()
    ens.close()
    # the batches run on streams of their own and overlap, so the roofline is
    # that of the whole graph-replayed step: the element kernels' algorithmic
    # bytes and flops (begin, stages, final: s launches a step) of every member
    # over the step time
    bts = sum(len(w["mesh"]["level"]) * element_stage_work(16, w["params"]["r"], 3, 1.0)[0] for w in mem) * stages
    fls = sum(len(w["mesh"]["level"]) * element_stage_work(16, w["params"]["r"], 3, 1.0)[1] for w in mem) * stages
    step_s = res["graph"] / steps
    roof = roofline(bts, fls, step_s, read_counters(os.path.join(ROOT, "profiles", "ensemble_64.traffic.json"),
                                                    stage_source_sha()),
                    "k_elem<r=1|2|3,P=16> of all batches, whole step")
    roof.update(scope="element kernels' algorithmic work per step over the step time (batches overlap)")
    return dict(workload="ensemble_64", members=len(mem), cells=cells, dofs_per_stage=dofs, steps=steps,
                value=dofs * stages * steps / res["graph"], unit="DoF-updates/s", roofline=roof,
                ms_per_step=res["graph"] / steps * 1e3, eager_ms_per_step=res["eager"] / steps * 1e3,
                one_by_one_ms_per_step=res["one_by_one"] / steps * 1e3,
                speedup_vs_one_by_one=res["one_by_one"] / res["graph"],
                graph_speedup_vs_eager=res["eager"] / res["graph"], autotuned=tuned)


def adjoint_bench(device, reps=3):
    """Gradient of the gauge misfit (adjoint_128: 128x128, r=2, 200 fixed-dt
    SSP3 steps, checkpoints every 20) w.r.t. per-cell Manning and bed offsets:
    forward and backward wall time and their ratio."""
    import torch
    from paper_2505_18743_amd import Solver
    from paper_2505_18743_amd.adjoint import PointObservation, observed_run
    from workloads import workload
    wl = workload("adjoint_128")
    s = Solver(wl["mesh"], wl["params"], device)
    xy = s.node_coords()
    s.set_bathymetry(wl["bed"](xy[:, 0], xy[:, 1]))
    dof = s.dof_coords()
    s.init_lake_at_rest(wl["eta0"](dof[:, 0], dof[:, 1]))
    state0 = [x.clone() for x in s.get_state()[:3]]
    K = s.n_cells
    dt = 0.9 * float(s.apply_operator(*state0)[4].cpu()[0])
    cells, phi = s.locate_points(wl["gauges"])
    obs = PointObservation(cells, phi, s.np_, device)
    nsteps, ck = int(wl["steps"]), int(wl["checkpoint_every"])
    zeros = torch.zeros(K, dtype=torch.float64, device=device)
    truth = observed_run(s, torch.as_tensor(wl["manning_truth"], device=device), zeros, state0, 0.0, dt, nsteps,
                         obs).detach()
    n0 = torch.as_tensor(wl["manning"], dtype=torch.float64, device=device)
    tf, tb, tp = [], [], []
    for rep in range(reps + 1):
        nman = n0.clone().requires_grad_(True)
        dbed = zeros.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = observed_run(s, nman, dbed, state0, 0.0, dt, nsteps, obs, checkpoint_every=ck)
        loss = ((out - truth) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.set_state(*state0)
        s.set_time(0.0)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        s.run(nsteps, dt)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if rep > 0:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
            tp.append(t4 - t3)
    s.sync()
    f, b, p = min(tf), min(tb), min(tp)
    return dict(workload="adjoint_128", cells=K, params=2 * K, steps=nsteps, checkpoint_every=ck,
                forward_ms=f * 1e3, backward_ms=b * 1e3, plain_forward_ms=p * 1e3,
                adjoint_over_forward=b / f, adjoint_over_plain_forward=b / p, loss=float(loss.detach()))


def imex_bench(steps, warmup, device):
    """The 256x256 beach dam break (Manning 0.025) stepped with the IMEX pair
    (RK32 explicit, TR-BDF2 for the friction) and, for reference, with the
    explicit RK32 scheme: DoF-updates/s per stage of each and the IMEX step's
    kernel-class shares."""
    import torch
    from workloads import workload
    out = {}
    for rk in ("imex", "rk32"):
        wl = workload("beach_dambreak_256")
        wl["params"] = dict(wl["params"], rk=rk)
        s, reset, _ = setup(wl, device)
        dofs_stage = 3 * (int(wl["params"]["r"]) + 1) ** 2 * s.n_cells
        s.run(warmup)
        s.sync()
        reset()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        s.run(steps)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        diag = s.diagnostics()
        out[rk] = dict(ms_per_step=ms / steps, value=dofs_stage * 3 * steps / (ms * 1e-3),
                       max_newton_it=diag["max_newton_it"], r0_cells=diag["n_r0_cells"])
        if rk == "imex":
            reset()
            torch.cuda.synchronize()
            s.profile(True)
            s.kernel_time_reset()
            ev0.record()
            s.run(steps)
            ev1.record()
            torch.cuda.synchronize()
            ms2 = ev0.elapsed_time(ev1)
            out[rk]["kernel_share"] = {k: round(v[0] / ms2, 4) for k, v in s.kernel_times().items()}
            s.profile(False)
        s.close()
    return dict(workload="beach_dambreak_256", steps=steps, unit="DoF-updates/s", **out)


# Wall times the paper reports for the static travelling vortex on its finest
# mesh (n_max = 5, 2N x N cells with N = 320), T = 1/6 s, 8 CPU processes
# (the table of the vortex section): scheme, r, seconds, DoFs (zeta + q).
PAPER_VORTEX = [("rk32", 1, 386.9, 2_457_600), ("ssp3", 2, 1516.0, 5_529_600), ("rk44", 3, 3658.0, 9_830_400)]


def vortex_bench(device, N=320):
    """The travelling vortex (Sec. 4.4) on 2N x N cells over [0, 2] x [0, 1],
    GLL rule with r + 2 nodes, exact state at the inflow, open outflow, walls,
    fixed dt = T / ceil(T / (0.9 x the positivity bound at t = 0))."""
    import numpy as np
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from exact import Vortex
    from workloads.gen import uniform_mesh_desc
    from paper_2505_18743_amd import Solver
    T = 1.0 / 6.0
    v = Vortex()
    out = []
    for rk, r, paper_s, paper_dofs in PAPER_VORTEX:
        progress(f"vortex {rk} r={r}")
        mesh = uniform_mesh_desc(2 * N, N, 0.0, 0.0, 1.0 / N, bc=("state", "open", "wall", "wall"))
        params = dict(r=r, S=(r + 2,), rule="gll", rk=rk, g=9.81, eps=1e-3, h_lim=0.0, eps0=1e-8, newton_max=20,
                      cfl=0.9, cfl_mode=1, tracer=False, tide=(0.0, 1.0, 0.0, 0.0), adapt_degree=False)
        s = Solver(mesh, params, device=device)
        s.set_bathymetry(np.zeros(s.n_vol))
        s.set_manning(np.zeros(s.n_cells))

        def given(x, y):
            h, u, w = v.fields(x, y, 0.0)
            return h - 0.0, h * u, h * w, np.zeros_like(x)
        s.set_boundary_state(given)
        d = s.dof_coords()
        h, u, w = v.fields(d[:, 0], d[:, 1], 0.0)
        st = [h, h * u, h * w]
        dtb = float(s.apply_operator(st[0], st[1], st[2], None, 0.0)[4].cpu()[0])
        n = int(math.ceil(T / (0.9 * dtb)))
        dt = T / n
        s.set_state(*st)
        s.run(3, dt)
        s.sync()
        s.set_state(*st)
        s.set_time(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(n, dt)
        s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        he, _, _ = v.fields(d[:, 0], d[:, 1], T)
        z = s.get_state()[0].cpu().numpy()
        err = float(np.sqrt(np.mean((z - he) ** 2)))
        dofs = 3 * (r + 1) ** 2 * s.n_cells
        out.append(dict(rk=rk, r=r, cells=s.n_cells, dofs=dofs, steps=n, dt=dt, wall_s=round(wall, 3),
                        rms_zeta_error=err, paper_wall_s=paper_s, paper_dofs=paper_dofs,
                        paper_hardware="8 CPU processes (deal.II, MPI), whole run"))
        s.close()
    return dict(workload="travelling_vortex_static_nmax5", T=T, runs=out)


# Table 7, with AMR at n_max = 5: wall time (s, 8 CPU processes) and DoFs
def react_work(S, r, M):
    """Algorithmic bytes and flops of the reaction kernel for one cell and
    M tracers on an S x S rule.  Bytes: the depth samples and zeta once, each
    tracer's concentration, the read and write of each tracer's residual R,
    the cell size.  Flops (sum factorisation, one lane a node row): the
    y-interpolated row coefficients of zeta and of each c_j, then per node the
    depth (an (r+1)-term interpolation, the weights and the mask) and per
    tracer c_j, w h c_j and its (r+1) x-projections, the y-projections of the
    (r+1)^2 row partials, and the M x M combination."""
    N1 = r + 1
    NP = N1 * N1
    nb = 8 * (S * S + NP + M * NP + 2 * M * NP + 1)
    fl = (2 * N1 * N1 * S + S * S * (2 * N1 + 4)
          + M * (2 * N1 * N1 * S + S * S * (4 * N1 + 1) + 2 * NP * S) + 2 * M * M * NP)
    return nb, fl


def tracers_bench(device, steps=20, M=3):
    """M tracers carried by the 256x256 beach flow (r=2, 16x16 samples, SSP3,
    fixed dt = the flow's first CFL step): the flow alone (sw_step), the flow
    recorded and the tracers replayed over it (sw_step_tracers), and the same
    with linear reactions between the tracers (sw_step_tracers_react, a
    conversion chain with feedback).  Tracer DoF-updates/s of both and the
    reaction kernel's launch time against its algorithmic bytes and flops."""
    import numpy as np
    import torch
    from paper_2505_18743_amd import Solver
    from workloads import workload
    wl = workload("beach_dambreak_256")
    flow, reset, bed = setup(wl, device)
    p = dict(wl["params"])
    p["tracer"] = True
    ctxs = []
    for _ in range(M):
        t = Solver(wl["mesh"], p, device=device)
        t.set_bathymetry(bed)
        t.set_manning(wl["manning"])
        ctxs.append(t)
    dof = flow.dof_coords()
    x = (dof[:, 0] - dof[:, 0].min()) / np.ptp(dof[:, 0])
    y = (dof[:, 1] - dof[:, 1].min()) / np.ptp(dof[:, 1])
    cs = [np.where(x < 0.5, 1.0, 0.2), 0.5 + 0.3 * np.cos(6.0 * y), 0.1 + 0.05 * np.sin(8.0 * (x + y))]
    cs = (cs * M)[:M]

    def restart():
        reset()
        st = flow.get_state()
        for t, c in zip(ctxs, cs):
            t.set_state(st[0], st[1], st[2], c)
            t.set_time(0.0)
    flow.step()
    flow.sync()
    dt = float(flow.diagnostics()["dt"])
    base = np.array([[-1.0, 0.0, 0.3], [0.8, -0.5, 0.0], [0.2, 0.5, -0.3]])
    B = np.zeros((M, M))
    B[:min(M, 3), :min(M, 3)] = base[:min(M, 3), :min(M, 3)]
    B = B * (0.01 / dt)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        restart()
        fn()
        fn()
        restart()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps
    ms_flow = timed(lambda: flow.step(dt))
    ms_plain = timed(lambda: flow.step_tracers(ctxs, dt))
    ms_react = timed(lambda: flow.step_tracers_react(ctxs, B, dt))
    # the reaction kernel's launches, timed with events on the library's stream
    restart()
    torch.cuda.synchronize()
    ctxs[0].profile(True, kinds=["reactions"])
    ctxs[0].kernel_time_reset()
    for _ in range(steps):
        flow.step_tracers_react(ctxs, B, dt)
    torch.cuda.synchronize()
    k_ms, k_n = ctxs[0].kernel_times()["reactions"]
    ctxs[0].profile(False)
    flow.sync()
    r = int(wl["params"]["r"])
    S = int(wl["params"]["S"][0])
    stages = {"fe": 1, "ssp3": 3, "rk32": 3, "rk44": 4}[wl["params"]["rk"]]
    K = flow.n_cells
    tdofs = M * (r + 1) ** 2 * K * stages
    nb, fl = react_work(S, r, M)
    launch_s = k_ms * 1e-3 / max(k_n, 1)
    gbs = nb * K / launch_s / 1e9
    tfl = fl * K / launch_s / 1e12
    for t in ctxs:
        t.close()
    flow.close()
    return dict(workload=f"beach_dambreak_256 flow + {M} tracers", cells=K, tracers=M, steps=steps, dt=dt,
                ms_per_step=dict(flow=round(ms_flow, 4), tracers=round(ms_plain, 4), reacting=round(ms_react, 4)),
                reaction_ms_per_step=round(ms_react - ms_plain, 4),
                tracer_value=dict(tracers=tdofs / ((ms_plain - ms_flow) * 1e-3),
                                  reacting=tdofs / ((ms_react - ms_flow) * 1e-3), unit="tracer DoF-updates/s"),
                react_kernel=dict(kernel=f"k_react<r={r},P={lanes_for(S)}> ({S}x{S} nodes, one lane a node row)",
                                  launches=k_n, us_per_launch=round(launch_s * 1e6, 2),
                                  algo_bytes_per_launch=nb * K, algo_flops_per_launch=fl * K,
                                  gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                                  tflops=round(tfl, 3), fp64_frac=round(tfl / FP64_PEAK_TFLOPS, 4)))


PAPER_VORTEX_AMR = [("rk32", 1, 74.1, 267_828), ("ssp3", 2, 286.7, 590_949), ("rk44", 3, 531.1, 1_028_256)]


def vortex_amr_bench(device, nmax=5, N=20, cases=None):
    """The travelling vortex with dynamic h-adaptivity as Sec. 4.4 runs it: the
    paper's quadrature (Table 1), initial mesh 2N x N, refinement to n_max
    levels on the vorticity indicator with theta_r = 1e-4, theta_c = 5e-5,
    a remesh every 5 steps, the initial mesh adapted n_max - 1 times to the
    initial state; beside it the static mesh of the finest level.  Both take
    the fixed dt = T / ceil(T / (0.9 x the static finest mesh's positivity
    bound at t = 0)); states are the exact solution at the support points.
    Wall times cover the whole run on the GPU (remeshes included); the AMR
    overhead is the time spent in sw_remesh."""
    import numpy as np
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from exact import Vortex
    from workloads.gen import uniform_mesh_desc
    from paper_2505_18743_amd import Solver
    T = 1.0 / 6.0
    v = Vortex()
    Nf = N * 2 ** (nmax - 1)
    grid = dict(x0=-1.0, y0=-1.0, dx=4.0, dy=3.0, b=np.zeros((2, 2)))
    out = []

    def inflow(x, y):
        h, u, w = v.fields(x, y, 0.0)
        return h, h * u, h * w, np.zeros_like(x)

    def exact_at_dofs(s):
        d = s.dof_coords()
        h, u, w = v.fields(d[:, 0], d[:, 1], 0.0)
        return [h, h * u, h * w]

    # Gauss-Lobatto weights on [0, 1] at the r + 1 support points
    gllw = {1: [0.5, 0.5], 2: [1 / 6, 2 / 3, 1 / 6], 3: [1 / 12, 5 / 12, 5 / 12, 1 / 12]}

    def l2_at_dofs(s, r, dx0):
        """L2 norm of the free-surface error at T by the support points' Lobatto
        rule (area-weighted, so meshes of different refinement compare)."""
        d = s.dof_coords()
        he, _, _ = v.fields(d[:, 0], d[:, 1], T)
        z = s.get_state()[0].cpu().numpy()
        lev = s.cells()[0]
        w1 = np.asarray(gllw[r])
        w = (np.outer(w1, w1).ravel()[None, :] * (dx0 / 2.0 ** lev[:, None]) ** 2).ravel()
        return float(np.sqrt(np.sum(w * (z - he) ** 2)))

    for rk, r, paper_s, paper_dofs in (cases or PAPER_VORTEX_AMR):
        params = dict(r=r, S=(r + 2,) * nmax, rule="gll", rk=rk, g=9.81, eps=1e-3, h_lim=0.0, eps0=1e-8,
                      newton_max=20, cfl=0.9, cfl_mode=1, tracer=False, tide=(0.0, 1.0, 0.0, 0.0),
                      adapt_degree=False, quadrature="paper")
        bc = ("state", "open", "wall", "wall")
        # static finest mesh
        progress(f"vortex static N={Nf} {rk} r={r}")
        st = Solver(uniform_mesh_desc(2 * Nf, Nf, 0.0, 0.0, 1.0 / Nf, bc=bc), dict(params, S=(r + 2,)),
                    device=device)
        st.set_bed_grid(grid)
        st.set_manning(np.zeros(st.n_cells))
        st.set_boundary_state(inflow)
        u0 = exact_at_dofs(st)
        dtb = float(st.apply_operator(*u0, None, 0.0)[4].cpu()[0])
        n = int(math.ceil(T / (0.9 * dtb)))
        dt = T / n
        st.set_state(*u0)
        st.run(3, dt)
        st.sync()
        st.set_state(*u0)
        st.set_time(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.run(n, dt)
        st.sync()
        torch.cuda.synchronize()
        wall_static = time.perf_counter() - t0
        err_static = l2_at_dofs(st, r, 1.0 / Nf)
        dofs_static = 3 * (r + 1) ** 2 * st.n_cells
        st.close()
        # adaptive run
        progress(f"vortex AMR n_max={nmax} {rk} r={r}")
        s = Solver(uniform_mesh_desc(2 * N, N, 0.0, 0.0, 1.0 / N, bc=bc), params, device=device)
        s.set_bed_grid(grid)
        s.set_manning(np.zeros(s.n_cells))
        s.set_boundary_state(inflow)
        s.set_state(*exact_at_dofs(s))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_remesh = 0.0
        n_remesh = 0
        dof_max = 0
        for _ in range(nmax - 1):
            s.remesh("vorticity", 1e-4, 5e-5, nmax)
            s.set_state(*exact_at_dofs(s))
        s.set_boundary_state(inflow)
        t_init = time.perf_counter() - t0
        k = 0
        while k < n:
            m = min(5, n - k)
            s.run(m, dt)
            k += m
            dof_max = max(dof_max, 3 * (r + 1) ** 2 * s.n_cells)
            if k < n:
                ta = time.perf_counter()
                st_r = s.remesh("vorticity", 1e-4, 5e-5, nmax)
                if not st_r["boundary_data_kept"]:   # the inflow side's faces changed
                    s.set_boundary_state(inflow)
                t_remesh += time.perf_counter() - ta
                n_remesh += 1
        s.sync()
        torch.cuda.synchronize()
        wall_amr = time.perf_counter() - t0
        out.append(dict(rk=rk, r=r, steps=n, dt=dt, remeshes=n_remesh,
                        static=dict(cells=dofs_static // (3 * (r + 1) ** 2), dofs=dofs_static,
                                    wall_s=round(wall_static, 3), l2_zeta_error=err_static),
                        amr=dict(dofs_final=3 * (r + 1) ** 2 * s.n_cells, dofs_max=dof_max,
                                 wall_s=round(wall_amr, 3), init_adapt_s=round(t_init, 3),
                                 remesh_s=round(t_remesh, 3), amr_overhead=round((t_remesh + t_init) / wall_amr, 4),
                                 l2_zeta_error=l2_at_dofs(s, r, 1.0 / N)),
                        speedup_amr_vs_static=round(wall_static / wall_amr, 3),
                        paper_amr_wall_s=paper_s, paper_amr_dofs=paper_dofs,
                        paper_hardware="8 CPU processes (deal.II, MPI), whole run"))
        s.close()
    return dict(workload=f"travelling_vortex_amr_nmax{nmax}", T=T, runs=out)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="beach_dambreak_256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ens-steps", type=int, default=300, help="ensemble_64 steps per mode (0: skip)")
    ap.add_argument("--ens-eager-only", action="store_true",
                    help="with --only ensemble: eager batched steps only (for a profiler)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint_128 gradient timing")
    ap.add_argument("--qt-steps", type=int, default=100, help="tidal_quadtree_r3 steps (0: skip)")
    ap.add_argument("--elem-wpb", type=int, default=0, help="wavefronts per workgroup of the fast element kernel "
                    "(0: library default)")
    ap.add_argument("--imex-steps", type=int, default=100, help="beach steps of the IMEX leg (0: skip)")
    ap.add_argument("--no-vortex", action="store_true", help="skip the travelling-vortex wall-time leg")
    ap.add_argument("--no-vortex-amr", action="store_true", help="skip the adaptive travelling-vortex leg")
    ap.add_argument("--no-tracers", action="store_true", help="skip the reacting-tracers leg")
    ap.add_argument("--only", choices=["ensemble", "adjoint", "quadtree", "imex", "vortex", "vortex_amr", "tracers"],
                    default=None,
                    help="run only that leg (for profiling it on its own); prints its JSON object")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs the hot path on a single MI355X "
              "and has no multi-GPU path (how it would shard is described in the design notes); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from workloads import workload
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (HIP device)", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    if args.only and args.calibrate_copy:
        calibration_copy(args.calibrate_copy, dev)
    if args.only == "ensemble":
        print(json.dumps(ensemble_bench(args.ens_steps, 3, dev, eager_only=args.ens_eager_only)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(adjoint_bench(dev)), flush=True)
        return
    if args.only == "quadtree":
        print(json.dumps(quadtree_bench(args.qt_steps, 3, dev)), flush=True)
        return
    if args.only == "imex":
        print(json.dumps(imex_bench(args.imex_steps, 3, dev)), flush=True)
        return
    if args.only == "vortex":
        print(json.dumps(vortex_bench(dev)), flush=True)
        return
    if args.only == "vortex_amr":
        print(json.dumps(vortex_amr_bench(dev)), flush=True)
        return
    if args.only == "tracers":
        print(json.dumps(tracers_bench(dev)), flush=True)
        return
    wl = workload(args.workload)
    s, reset, _ = setup(wl, dev)
    if args.elem_wpb:
        s.set_workgroup(args.elem_wpb)
    stages = {"fe": 1, "ssp3": 3, "rk32": 3, "rk44": 4}[wl["params"]["rk"]]
    r = int(wl["params"]["r"])
    S = int(wl["params"]["S"][0])
    nf = 3 + (1 if wl["params"]["tracer"] else 0)
    dofs_stage = nf * (r + 1) ** 2 * s.n_cells

    progress(f"{args.workload}: warm-up")
    s.run(args.warmup)
    s.sync()
    reset()
    s.sync()
    if args.calibrate_copy:
        calibration_copy(args.calibrate_copy, dev)
    progress(f"{args.workload}: timed regions")
    # timed region 1: the whole step with no per-kernel events -> value
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    s.run(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s.sync()
    diag = s.diagnostics()
    value = dofs_stage * stages * args.steps / (ms * 1e-3)

    # timed region 2: the same steps from the same start, HIP events (on the
    # library's stream) around the dominant kernel's launches only
    reset()
    torch.cuda.synchronize()
    s.profile(True, kinds=["element_stage"])
    s.kernel_time_reset()
    ev0.record()
    s.run(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms2 = ev0.elapsed_time(ev1)
    kt = s.kernel_times()
    s.profile(False)

    # region 3: every kernel class timed (shares of the step, informational)
    reset()
    n3 = min(args.steps, 100)
    torch.cuda.synchronize()
    s.profile(True)
    s.kernel_time_reset()
    ev0.record()
    s.run(n3)
    ev1.record()
    torch.cuda.synchronize()
    ms3 = ev0.elapsed_time(ev1)
    kt3 = s.kernel_times()
    s.profile(False)
    s.sync()

    # dominant kernel: the fast element kernel of stages 2..s
    k_ms, k_n = kt["element_stage"]
    avg_s = (k_ms / max(k_n, 1)) * 1e-3
    # stages 2..s combine 1..s-1 stored residuals: average
    mean_terms = sum(range(1, stages)) / max(stages - 1, 1)
    bpc, fpc = element_stage_work(S, r, nf, mean_terms)
    roof = roofline(bpc * s.n_cells, fpc * s.n_cells, avg_s, read_counters(TRAFFIC_FILE, stage_source_sha()),
                    f"k_elem<r={r},P={lanes_for(S)},F_STAGE>")
    roof.update(launches=k_n, timed_region_ms=round(ms2, 3),
                kernel_share={k: round(v[0] / ms3, 4) for k, v in kt3.items()})
    # (not in counter runs: their own calibration copies must be the only ones)
    if not args.calibrate_copy:
        copy_gbs = copy_roof(dev)
        gbs = roof["algo_bytes_per_launch"] / avg_s / 1e9
        roof.update(copy_gbs=round(copy_gbs, 1), hbm_frac_of_copy=round(gbs / copy_gbs, 4))
    line = dict(metric="FP64 DoF-updates/s per RK stage", value=value, unit="DoF-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload=args.workload, cells=s.n_cells, r=r, S=S, rk=wl["params"]["rk"],
                            stages_per_step=stages, dofs_per_stage=dofs_stage, parallelism="single GPU"),
                roofline=roof)
    line["config"]["max_newton_it"] = diag["max_newton_it"]
    line["config"]["r0_cells"] = diag["n_r0_cells"]
    # the paper's DoF count with degree-0 cells as one dof per field (their
    # number at the end of the timed steps)
    nr0 = int(diag["n_r0_cells"])
    active = nf * ((r + 1) ** 2 * (s.n_cells - nr0) + nr0)
    line["active"] = dict(dofs_per_stage=active, value=active * stages * args.steps / (ms * 1e-3),
                          unit="DoF-updates/s")
    if args.qt_steps > 0:
        progress("quadtree")
        line["quadtree"] = quadtree_bench(args.qt_steps, 3, dev)
    if args.ens_steps > 0:
        progress("ensemble")
        line["ensemble"] = ensemble_bench(args.ens_steps, 3, dev)
    if not args.no_adjoint:
        progress("adjoint")
        line["adjoint"] = adjoint_bench(dev)
    if args.imex_steps > 0:
        progress("imex")
        line["imex"] = imex_bench(args.imex_steps, 3, dev)
    if not args.no_vortex:
        progress("vortex")
        line["vortex"] = vortex_bench(dev)
    if not args.no_vortex_amr:
        line["vortex_amr"] = vortex_amr_bench(dev)
    if not args.no_tracers:
        progress("reacting tracers")
        line["tracers"] = tracers_bench(dev)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle on the host)")
        line["cpu_baseline"] = cpu_baseline(args.workload)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
