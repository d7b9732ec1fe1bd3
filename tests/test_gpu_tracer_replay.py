"""GPU: tracer steps that replay a recorded flow (sw_step_record with the end
state, then sw_tracer_step).

The flow does not depend on the tracer, and the replay runs the coupled
step's tracer solve and residuals on the recorded flow, so a replay of a
record made with a tracer reproduces the coupled tracer bit for bit, for any
initial tracer; the coupled run is tied to the oracle here again.  A record
of a flow-only context (other element kernel, other summation order) gives
the tracer within the step tolerance.
"""
import numpy as np
import pytest
import torch

from test_gpu_parity import TOL_STEP, cpu, gpu_from_oracle, hanging_case, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def fixed_dt(s, st):
    dtb = s.apply_operator(st[0], st[1], st[2], st[3], 0.0)[4]
    return 0.3 * float(dtb.cpu()[0])


def record(s, st, dt, n):
    ns = s.n_stages()
    stages = torch.empty(n, ns, 3, s.n_dofs, dtype=torch.float64, device="cuda:0")
    end = torch.empty(n, 3, s.n_dofs, dtype=torch.float64, device="cuda:0")
    s.set_state(*st)
    s.set_time(0.0)
    r0 = 0
    for k in range(n):
        s.step_record(dt, stages[k], end[k])
        r0 = max(r0, s.diagnostics()["n_r0_cells"])
    s.sync()
    return stages, end, r0


def replay(s, st, stages, end, dt):
    s.set_state(*st)
    s.set_time(0.0)
    for k in range(stages.shape[0]):
        s.tracer_step(stages[k], end[k], dt)
    s.sync()
    return s.get_state()


@pytest.mark.parametrize("rk", ["ssp3", "rk32", "fe", "imex"])
def test_replay_equals_coupled_and_oracle(rk):
    say(f"case: tracer replay, hanging mesh + tide, {rk}, 12 steps, two tracers")
    o, b = hanging_case(2, (16, 8))
    o.p.rk = rk
    st0 = o.get_state()
    rec = gpu_from_oracle(o, b)
    dt = fixed_dt(rec, st0)
    n = 12
    stages, end, r0 = record(rec, st0, dt, n)
    coupled = rec.get_state()
    say(f"  dt {dt:.4e}, cells of degree 0 up to {r0}")
    # replay with the recorded tracer: the same tracer and flow, bit for bit
    rep = gpu_from_oracle(o, b)
    got = replay(rep, st0, stages, end, dt)
    for f in range(4):
        assert torch.equal(got[f], coupled[f]), ("field", f, float((got[f] - coupled[f]).abs().max()))
    da, db = rep.diagnostics(), rec.diagnostics()
    assert da["t"] == db["t"] and da["dt"] == db["dt"]
    assert da["total_mass"] == pytest.approx(db["total_mass"], rel=1e-13)
    # a replay forms no flow target and takes no Newton step
    assert da["n_pos_viol"] == 0 and da["min_target_mass"] == 1e300 and da["max_newton_it"] == 0
    # a second tracer over the same record equals its coupled run
    dof = o.dof_coords()
    c1 = np.where(dof[..., 0] < 1300.0, 1.0, 0.25) + 0.1 * np.sin(dof[..., 1] / 200.0)
    st1 = [st0[0], st0[1], st0[2], c1]
    got1 = replay(rep, st1, stages, end, dt)
    rec.set_state(*st1)
    rec.set_time(0.0)
    for _ in range(n):
        rec.step(dt)
    rec.sync()
    ref1 = rec.get_state()
    assert torch.equal(got1[3], ref1[3]), float((got1[3] - ref1[3]).abs().max())
    # the oracle's coupled steps with the same dt
    o.state[3] = torch.as_tensor(c1)
    for _ in range(n):
        o.step(dt)
    K = o.m.K
    e = rel(cpu(got1[3], K), o.get_state()[3])
    say(f"  replayed tracer vs oracle rel err {e:.3e}")
    assert e < TOL_STEP
    rec.close()
    rep.close()


def test_coupled_steps_after_a_replay():
    say("case: coupled SSP3 steps on a context right after 12 replayed steps, against the recording run")
    o, b = hanging_case(2, (16, 8))
    st0 = o.get_state()
    rec = gpu_from_oracle(o, b)
    dt = fixed_dt(rec, st0)
    stages, end, _ = record(rec, st0, dt, 12)
    rep = gpu_from_oracle(o, b)
    replay(rep, st0, stages, end, dt)
    # the replay leaves the flow's volume terms of the next start out; the
    # next coupled step prepares that start again
    for _ in range(4):
        rec.step(dt)
        rep.step(dt)
    rec.sync()
    rep.sync()
    K = o.m.K
    a, c = rep.get_state(), rec.get_state()
    for f, name in enumerate(("eta", "qx", "qy", "c")):
        e = rel(cpu(a[f], K), cpu(c[f], K))
        say(f"  {name} rel diff {e:.3e}")
        assert e < 1e-13
    rec.close()
    rep.close()


def test_replay_of_a_flow_only_record():
    say("case: tracer replay of a record made without a tracer (fast element kernel), 10 SSP3 steps")
    o, b = hanging_case(2, (16, 8))
    st0 = o.get_state()
    o.p.tracer = False
    flow = gpu_from_oracle(o, b)
    o.p.tracer = True
    rep = gpu_from_oracle(o, b)
    dt = fixed_dt(rep, st0)
    n = 10
    stages, end, _ = record(flow, st0[:3], dt, n)
    got = replay(rep, st0, stages, end, dt)
    for _ in range(n):
        o.step(dt)
    K = o.m.K
    for f, name in enumerate(("eta", "qx", "qy", "c")):
        e = rel(cpu(got[f], K), o.get_state()[f])
        say(f"  {name} rel err vs oracle {e:.3e}")
        assert e < TOL_STEP
    flow.close()
    rep.close()


def test_tracer_step_argument_errors():
    say("case: tracer_step argument checks")
    o, b = hanging_case(1, (8, 4), tracer=False)
    s = gpu_from_oracle(o, b)
    st = torch.zeros(3, 3, s.n_dofs, dtype=torch.float64, device="cuda:0")
    end = torch.zeros(3, s.n_dofs, dtype=torch.float64, device="cuda:0")
    with pytest.raises(RuntimeError, match="tracer"):
        s.tracer_step(st, end, 1.0)
    with pytest.raises(ValueError):
        s.tracer_step(st[:2], end, 1.0)
    s.close()
