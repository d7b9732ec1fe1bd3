"""GPU: tracers that react with each other (sw_step_tracers_react: the
source h phi_k(c_1, ..., c_M) of eq:shw with phi_k = sum_j B_kj c_j, taken
explicitly in every stage as eq:imex_shw takes it) against the oracle's
stage-by-stage coupled step (oracle.step_coupled).

* 12 steps of three tracers on the hanging quadtree with wet/dry cells, tide
  and Manning friction (r = 2, SSP3; r = 1, IMEX), with a non-symmetric B
  that converts and feeds back, and one tracer with its own diffusion and
  decay: every tracer within the step tolerance of the oracle's;
* the same with the paper's quadrature (Table 1), whose volume rule carries
  the reaction integrals;
* B = 0 equals sw_step_tracers bit for bit (the stage-by-stage order
  changes nothing else), and the flow context's own state is untouched by
  the reactions;
* tracer contexts on streams other than the flow's give the same tracers
  bit for bit (the call orders them with events);
* the largest set the call takes (eight tracers, a random B) and a single
  tracer reacting with itself, against the oracle;
* at full size (the 256x256 beach, the benchmark's launch configuration),
  B = -kappa I equals each tracer context's own decay to 1e-12;
* argument checks: more than eight tracers, a context listed twice, a
  non-finite entry.
"""
import numpy as np
import pytest
import torch

from oracle import step_coupled
from test_gpu_parity import TOL_STEP, cpu, gpu_from_oracle, hanging_case, rel
from test_gpu_paper_quadrature import coastal_paper
from test_gpu_tracer_replay import fixed_dt
from test_gpu_tracer_sources import with_sources

pytestmark = pytest.mark.gpu

BASE = np.array([[-1.0, 0.0, 0.3],
                 [0.8, -0.5, 0.0],
                 [0.2, 0.5, -0.3]])
SOURCES = [dict(tracer_diff=0.33, tracer_strain=0.004, tracer_decay=1e-4), dict(), dict()]


def say(*a):
    print(*a, flush=True)


def inits(o):
    d = o.dof_coords()
    x, y = d[..., 0], d[..., 1]
    return [np.where(x < 1300.0, 1.0, 0.25) + 0.1 * np.sin(y / 200.0),
            0.5 + 0.3 * np.cos(x / 300.0),
            0.2 + 0.1 * np.sin((x + y) / 250.0)]


def run_pair(make, nsteps=12, rk=None):
    o, b = make()
    if rk:
        o.p.rk = rk
    st0 = o.get_state()
    flow = gpu_from_oracle(o, b)
    dt = fixed_dt(flow, st0)
    B = BASE * (0.02 / dt)           # a few per cent of each tracer reacts per step
    cs = inits(o)
    oracles, ctxs = [], []
    for src, c in zip(SOURCES, cs):
        oi, _ = make()
        if rk:
            oi.p.rk = rk
        with_sources(oi, **src)
        ctxs.append(gpu_from_oracle(oi, b))
        oi.set_state(st0[0], st0[1], st0[2], c)
        oracles.append(oi)
    flow.set_state(*st0)
    flow.set_time(0.0)
    for t, c in zip(ctxs, cs):
        t.set_state(st0[0], st0[1], st0[2], c)
        t.set_time(0.0)
    for _ in range(nsteps):
        flow.step_tracers_react(ctxs, B, dt)
        step_coupled(oracles, B, dt)
    flow.sync()
    K = o.m.K
    for k, (t, oi) in enumerate(zip(ctxs, oracles)):
        got = t.get_state()
        e = rel(cpu(got[3], K), oi.adapted_state()[3])
        moved = rel(cpu(got[3], K), np.asarray(cs[k]))
        say(f"  tracer {k}: rel err vs oracle {e:.3e} (change over the run {moved:.3e})")
        assert e < TOL_STEP, (k, e)
        assert moved > 1e-2
        t.close()
    flow.close()


def test_reacting_tracers_ssp3_r2():
    say("case: 3 reacting tracers, hanging mesh r=2 S=(16,8), SSP3, 12 steps")
    run_pair(lambda: hanging_case(2, (16, 8)))


def test_reacting_tracers_imex_r1():
    say("case: 3 reacting tracers, hanging mesh r=1 S=(8,4), IMEX, 12 steps")
    run_pair(lambda: hanging_case(1, (8, 4)), rk="imex")


def test_reacting_tracers_paper_quadrature():
    say("case: 3 reacting tracers, paper quadrature r=2, SSP3, 8 steps")
    run_pair(lambda: coastal_paper(2), nsteps=8)


def test_eight_reacting_tracers_and_one():
    say("case: the largest set (8 reacting tracers) and a single tracer reacting with itself, r=1, 4 steps")
    o, b = hanging_case(1, (8, 4))
    st0 = o.get_state()
    flow = gpu_from_oracle(o, b)
    dt = fixed_dt(flow, st0)
    rng = np.random.default_rng(8)
    d = o.dof_coords()
    K = o.m.K
    for M in (8, 1):
        B = rng.uniform(-1.0, 1.0, (M, M)) * (0.02 / dt)
        cs = [0.5 + 0.4 * np.sin((k + 1) * d[..., 0] / 500.0) * np.cos(d[..., 1] / 400.0) for k in range(M)]
        oracles, ctxs = [], []
        for c in cs:
            oi, _ = hanging_case(1, (8, 4))
            ctxs.append(gpu_from_oracle(oi, b))
            oi.set_state(st0[0], st0[1], st0[2], c)
            oracles.append(oi)
        flow.set_state(*st0)
        flow.set_time(0.0)
        for t, c in zip(ctxs, cs):
            t.set_state(st0[0], st0[1], st0[2], c)
            t.set_time(0.0)
        for _ in range(4):
            flow.step_tracers_react(ctxs, B, dt)
            step_coupled(oracles, B, dt)
        flow.sync()
        worst = 0.0
        for t, oi in zip(ctxs, oracles):
            worst = max(worst, rel(cpu(t.get_state()[3], K), oi.adapted_state()[3]))
            t.close()
        say(f"  M={M}: worst tracer rel err vs oracle {worst:.3e}")
        assert worst < TOL_STEP
    flow.close()


def test_zero_reactions_equal_step_tracers():
    say("case: B = 0 equals sw_step_tracers bit for bit, 6 steps")
    o, b = hanging_case(2, (16, 8))
    st0 = o.get_state()
    cs = inits(o)
    results = []
    for react in (True, False):
        flow = gpu_from_oracle(o, b)
        dt = fixed_dt(flow, st0)
        ctxs = []
        for src, c in zip(SOURCES, cs):
            oi, _ = hanging_case(2, (16, 8))
            t = gpu_from_oracle(with_sources(oi, **src), b)
            t.set_state(st0[0], st0[1], st0[2], c)
            t.set_time(0.0)
            ctxs.append(t)
        flow.set_state(*st0)
        flow.set_time(0.0)
        for _ in range(6):
            if react:
                flow.step_tracers_react(ctxs, np.zeros((3, 3)), dt)
            else:
                flow.step_tracers(ctxs, dt)
        flow.sync()
        results.append(([t.get_state() for t in ctxs], flow.get_state()))
        for t in ctxs:
            t.close()
        flow.close()
    (a, fa), (b_, fb) = results
    for f in range(4):
        assert torch.equal(fa[f], fb[f]), f
    for ga, gb in zip(a, b_):
        for f in range(4):
            assert torch.equal(ga[f], gb[f]), f


def test_reacting_tracers_on_streams_of_their_own():
    say("case: 3 reacting tracers whose contexts live on two other streams and the flow's, 6 steps, "
        "against all on the flow's stream")
    o, b = hanging_case(2, (16, 8))
    st0 = o.get_state()
    cs = inits(o)
    extra = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority

    def run(streams):
        flow = gpu_from_oracle(o, b)
        dt = fixed_dt(flow, st0)
        B = BASE * (0.02 / dt)
        ctxs = []
        for src, c, sm in zip(SOURCES, cs, streams):
            with torch.cuda.stream(sm):
                oi, _ = hanging_case(2, (16, 8))
                t = gpu_from_oracle(with_sources(oi, **src), b)
                t.set_state(st0[0], st0[1], st0[2], c)
                t.set_time(0.0)
            ctxs.append(t)
        flow.set_state(*st0)
        flow.set_time(0.0)
        for _ in range(6):
            flow.step_tracers_react(ctxs, B, dt)
        out = []
        for t, sm in zip(ctxs, streams):
            with torch.cuda.stream(sm):
                out.append(t.get_state()[3].clone())
            sm.synchronize()
            t.close()
        flow.close()
        return out

    cur = torch.cuda.current_stream()
    a = run([cur, cur, cur])
    bb = run([extra[0], cur, extra[1]])
    for k, (x, y) in enumerate(zip(a, bb)):
        assert torch.equal(x, y), (k, float((x - y).abs().max()))


def test_full_size_diagonal_reactions_are_each_tracers_decay():
    say("case: beach_dambreak_256 at full size, 3 tracers, B = -kappa I against each context's own decay, 5 steps")
    from paper_2505_18743_amd import Solver
    from workloads import workload
    wl = workload("beach_dambreak_256")
    p = dict(wl["params"])
    p["tracer"] = True
    flow = Solver(wl["mesh"], wl["params"], device="cuda:0")
    xy = flow.node_coords()
    bed = wl["bed"](xy[:, 0], xy[:, 1])
    dof = flow.dof_coords()
    eta0 = wl["eta0"](dof[:, 0], dof[:, 1])

    def ctx(pp):
        s = Solver(wl["mesh"], pp, device="cuda:0")
        s.set_bathymetry(bed)
        s.set_manning(wl["manning"])
        return s
    flow.set_bathymetry(bed)
    flow.set_manning(wl["manning"])
    flow.init_lake_at_rest(eta0)
    st0 = flow.get_state()
    flow.step()
    dt = float(flow.diagnostics()["dt"])
    kappa = 0.01 / dt
    x = (dof[:, 0] - dof[:, 0].min()) / np.ptp(dof[:, 0])
    cs = [np.where(x < 0.5, 1.0, 0.2), 0.5 + 0.3 * np.cos(6.0 * x), 0.1 + 0.05 * np.sin(8.0 * x)]
    pd = dict(p, tracer_decay=kappa)
    results = []
    for react in (True, False):
        ctxs = [ctx(p if react else pd) for _ in cs]
        flow.set_state(st0[0], st0[1], st0[2])
        flow.set_time(0.0)
        for t, c in zip(ctxs, cs):
            t.set_state(st0[0], st0[1], st0[2], c)
            t.set_time(0.0)
        for _ in range(5):
            if react:
                flow.step_tracers_react(ctxs, -kappa * np.eye(3), dt)
            else:
                flow.step_tracers(ctxs, dt)
        flow.sync()
        results.append([t.get_state()[3].cpu().numpy() for t in ctxs])
        for t in ctxs:
            t.close()
    flow.close()
    for k, (a, b) in enumerate(zip(*results)):
        e = rel(a, b)
        moved = rel(b, cs[k])
        say(f"  tracer {k}: reactions vs own decay rel diff {e:.3e} (change over the run {moved:.3e})")
        assert e < 1e-12 and moved > 1e-3


def test_react_argument_checks():
    say("case: sw_step_tracers_react argument checks")
    o, b = hanging_case(1, (8, 4))
    flow = gpu_from_oracle(o, b)
    t1 = gpu_from_oracle(hanging_case(1, (8, 4))[0], b)
    dt = 1.0
    with pytest.raises(RuntimeError, match="twice"):
        flow.step_tracers_react([t1, t1], np.zeros((2, 2)), dt)
    with pytest.raises(RuntimeError, match="not finite"):
        flow.step_tracers_react([t1], np.array([[np.nan]]), dt)
    with pytest.raises(RuntimeError, match="1 to 8"):
        flow.step_tracers_react([t1] * 9, np.zeros((9, 9)), dt)
    with pytest.raises(RuntimeError, match="flow"):
        flow.step_tracers_react([flow], np.zeros((1, 1)), dt)
    t1.close()
    flow.close()
