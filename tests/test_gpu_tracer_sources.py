"""GPU: the tracer's numerical diffusion (eq:numdiff, nu_K = C |K| S / r^2)
and first-order decay source (the reaction h phi(c), phi = -kappa c, of
eq:shw) against the oracle: the tracer residual of one evaluation on the
hanging quadtree mesh (r = 1, 2, 3), 20 coupled steps (SSP3 and IMEX), and
further tracers, each with its own diffusion and decay, carried over one
recorded flow by contexts of their own (sw_tracer_step): several tracers
on one flow, each equal to its coupled run bit for bit and to the oracle.
Several tracer contexts stepped by one call (sw_step_tracers, launch groups
of up to eight) over a flooding shore, where cells change degree, equal
their coupled runs bit for bit too.
"""
import numpy as np
import pytest
import torch

from test_gpu_parity import TOL_RHS, TOL_STEP, compare_states, cpu, gpu_from_oracle, hanging_case, rel
from test_gpu_tracer_replay import fixed_dt, record, replay

pytestmark = pytest.mark.gpu

SRC = dict(tracer_diff=0.33, tracer_strain=0.004, tracer_decay=2e-3)


def say(*a):
    print(*a, flush=True)


def with_sources(o, **src):
    for k, v in src.items():
        setattr(o.p, k, v)
    return o


@pytest.mark.parametrize("r,S", [(1, (8, 4)), (2, (16, 8)), (3, (16, 8, 5))])
def test_apply_operator_tracer_sources(r, S):
    say(f"case: tracer residual with diffusion and decay, hanging mesh r={r} S={S}")
    o, b = hanging_case(r, S)
    with_sources(o, **SRC)
    s = gpu_from_oracle(o, b)
    rng = np.random.default_rng(30 + r)
    st = o.get_state()
    st = [st[0], rng.uniform(-0.5, 0.5, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape),
          st[3] + 0.2 * rng.uniform(-1, 1, st[0].shape)]
    F, Gx, Gy, R, _ = o.apply_operator(st, 700.0)
    g = s.apply_operator(st[0], st[1], st[2], st[3], 700.0)
    s.sync()
    K = o.m.K
    # the sources are a sizeable part of R
    o0, _ = hanging_case(r, S)
    R0 = o0.apply_operator(st, 700.0)[3]
    assert np.abs(R - R0).max() > 1e-3 * np.abs(R).max()
    for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy), ("R", g[3], R)):
        e = rel(cpu(gg, K), rr)
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_RHS, (name, e)
    s.close()


@pytest.mark.parametrize("rk", ["ssp3", "imex"])
def test_steps_tracer_sources(rk):
    say(f"case: 20 {rk} steps, hanging mesh + tide + tracer with diffusion and decay")
    o, b = hanging_case(2, (16, 8))
    o.p.rk = rk
    with_sources(o, **SRC)
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    for _ in range(20):
        o.step()
        s.step()
    s.sync()
    compare_states(o, s, TOL_STEP, "20 steps")
    s.close()


def test_several_tracers_over_one_recorded_flow():
    say("case: one flow recorded (tracer without sources), two more tracers with their own sources replayed")
    o, b = hanging_case(2, (16, 8))
    st0 = o.get_state()
    rec = gpu_from_oracle(o, b)
    dt = fixed_dt(rec, st0)
    n = 12
    stages, end, _ = record(rec, st0, dt, n)
    dof = o.dof_coords()
    tracers = [(dict(tracer_diff=0.33, tracer_strain=0.004, tracer_decay=0.0),
                np.where(dof[..., 0] < 1300.0, 1.0, 0.25) + 0.1 * np.sin(dof[..., 1] / 200.0)),
               (dict(tracer_diff=0.0, tracer_strain=0.0, tracer_decay=5e-3), 0.5 + 0.3 * np.cos(dof[..., 0] / 300.0))]
    K = o.m.K
    for src, c in tracers:
        oi, _ = hanging_case(2, (16, 8))
        with_sources(oi, **src)
        rep = gpu_from_oracle(oi, b)
        st = [st0[0], st0[1], st0[2], c]
        got = replay(rep, st, stages, end, dt)
        # its coupled run on the GPU, bit for bit
        rep.set_state(*st)
        rep.set_time(0.0)
        for _ in range(n):
            rep.step(dt)
        rep.sync()
        ref = rep.get_state()
        assert torch.equal(got[3], ref[3]), (src, float((got[3] - ref[3]).abs().max()))
        # and the oracle's coupled run with the same sources
        oi.state[3] = torch.as_tensor(c)
        for _ in range(n):
            oi.step(dt)
        e = rel(cpu(got[3], K), oi.adapted_state()[3])
        say(f"  sources {src}: replayed tracer vs oracle rel err {e:.3e}")
        assert e < TOL_STEP
        rep.close()
    rec.close()


def flooding_case():
    """The hanging mesh with a 0.6 m bump on the shore: cells flood and dry
    within a few steps at 0.8 of the first step's bound (on the oracle, the
    degree-0 count goes 25, 25, 25, 26, 25, 26, ...), so a replay's final
    combination takes both the cells that keep their degree and those that
    change it."""
    o, b = hanging_case(2, (16, 8))
    dof = o.dof_coords()
    o.init_lake_at_rest(0.6 * np.exp(-((dof[..., 0] - 1400.0) ** 2 + (dof[..., 1] - 1000.0) ** 2) / 200.0 ** 2))
    return o, b


def flooding_dt(s, st):
    return 0.8 * float(s.apply_operator(st[0], st[1], st[2], st[3], 0.0)[4].cpu()[0])


def test_replay_with_degree_changes():
    say("case: sw_tracer_step over a flooding shore, 12 steps, against the coupled run")
    o, b = flooding_case()
    st0 = o.get_state()
    rec = gpu_from_oracle(o, b)
    dt = flooding_dt(rec, st0)
    n = 12
    ns = rec.n_stages()
    stages = torch.empty(n, ns, 3, rec.n_dofs, dtype=torch.float64, device="cuda:0")
    end = torch.empty(n, 3, rec.n_dofs, dtype=torch.float64, device="cuda:0")
    rec.set_state(*st0)
    rec.set_time(0.0)
    r0 = []
    for k in range(n):
        rec.step_record(dt, stages[k], end[k])
        r0.append(rec.diagnostics()["n_r0_cells"])
    rec.sync()
    say(f"  dt {dt:.4e}, degree-0 cells after each step: {r0}")
    assert len(set(r0)) > 1, r0
    dof = o.dof_coords()
    oi, _ = flooding_case()
    rep = gpu_from_oracle(with_sources(oi, tracer_diff=0.33, tracer_strain=0.004, tracer_decay=2e-3), b)
    st = [st0[0], st0[1], st0[2], 0.5 + 0.3 * np.cos(dof[..., 0] / 300.0)]
    got = replay(rep, st, stages, end, dt)
    rep.set_state(*st)
    rep.set_time(0.0)
    for _ in range(n):
        rep.step(dt)
    rep.sync()
    ref = rep.get_state()
    for f in range(4):
        assert torch.equal(got[f], ref[f]), (f, float((got[f] - ref[f]).abs().max()))
    rep.close()
    rec.close()


def test_step_tracers_one_call():
    say("case: sw_step_tracers over a flooding shore, a flow context with its own tracer and two more tracers, 12 steps")
    o, b = flooding_case()
    st0 = o.get_state()
    flow = gpu_from_oracle(o, b)
    dt = flooding_dt(flow, st0)
    dof = o.dof_coords()
    srcs = [dict(tracer_diff=0.33, tracer_strain=0.004, tracer_decay=0.0),
            dict(tracer_diff=0.0, tracer_strain=0.0, tracer_decay=5e-3)]
    inits = [np.where(dof[..., 0] < 1300.0, 1.0, 0.25), 0.5 + 0.3 * np.cos(dof[..., 0] / 300.0)]
    ctxs = []
    for src in srcs:
        oi, _ = flooding_case()
        ctxs.append(gpu_from_oracle(with_sources(oi, **src), b))
    flow.set_state(*st0)
    flow.set_time(0.0)
    for t, c in zip(ctxs, inits):
        t.set_state(st0[0], st0[1], st0[2], c)
        t.set_time(0.0)
    n = 12
    r0 = []
    for _ in range(n):
        flow.step_tracers(ctxs, dt)
        r0.append(flow.diagnostics()["n_r0_cells"])
    flow.sync()
    say(f"  degree-0 cells after each step: {r0}")
    # cells change degree, so the final combination runs both the shared
    # tracer kernel and each context's general kernel
    assert len(set(r0)) > 1, r0
    got = [t.get_state() for t in ctxs]
    # the flow itself equals its plain coupled run; each tracer its own coupled run
    ref = gpu_from_oracle(o, b)
    ref.set_state(*st0)
    for _ in range(n):
        ref.step(dt)
    ref.sync()
    for f in range(4):
        assert torch.equal(flow.get_state()[f], ref.get_state()[f]), f
    for t, c, g in zip(ctxs, inits, got):
        t.set_state(st0[0], st0[1], st0[2], c)
        t.set_time(0.0)
        for _ in range(n):
            t.step(dt)
        t.sync()
        own = t.get_state()
        for f in range(4):
            assert torch.equal(g[f], own[f]), f
        t.close()
    with pytest.raises(RuntimeError, match="flow"):
        flow.step_tracers([flow], dt)
    flow.close()
    ref.close()


def test_step_tracers_two_launch_groups():
    say("case: sw_step_tracers with ten tracer contexts (launch groups of eight and two) over a flooding shore, 6 steps")
    o, b = flooding_case()
    st0 = o.get_state()
    flow = gpu_from_oracle(o, b)
    dt = flooding_dt(flow, st0)
    dof = o.dof_coords()
    ctxs, inits = [], []
    for i in range(10):
        oi, _ = flooding_case()
        src = dict(tracer_diff=0.1 * (i % 3), tracer_strain=0.004, tracer_decay=1e-3 * i)
        ctxs.append(gpu_from_oracle(with_sources(oi, **src), b))
        inits.append(0.5 + 0.3 * np.cos(dof[..., 0] / (200.0 + 30.0 * i)))
    flow.set_state(*st0)
    flow.set_time(0.0)
    for t, c in zip(ctxs, inits):
        t.set_state(st0[0], st0[1], st0[2], c)
        t.set_time(0.0)
    n = 6
    for _ in range(n):
        flow.step_tracers(ctxs, dt)
    flow.sync()
    got = [t.get_state()[3].clone() for t in ctxs]
    # each tracer equals its own coupled run, in either launch group
    for i, (t, c, g) in enumerate(zip(ctxs, inits, got)):
        t.set_state(st0[0], st0[1], st0[2], c)
        t.set_time(0.0)
        for _ in range(n):
            t.step(dt)
        t.sync()
        own = t.get_state()[3]
        assert torch.equal(g, own), (i, float((g - own).abs().max()))
        t.close()
    flow.close()
