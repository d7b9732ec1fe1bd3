"""GPU: the IMEX step (explicit RK32 companion, TR-BDF2 companion for the
Manning friction, linearised at the previous stage; Sec. 3.1,
eq:algebraic_discharge, eq:mass_matrix_discharge, Appendix A) against the
oracle, element by element:

* windows of the 256x256 beach case with Manning friction: the dam line, and
  the shoreline with a surge flooding dry cells (degree-0 cells and their
  scalar update);
* the hanging quadtree mesh with a tracer, the elevation boundary and Manning
  friction at r = 2 and r = 3;
* a uniform flow on a flat periodic bed under stiff friction (kappa q0 dt =
  12), where the explicit step diverges: GPU against the oracle step by step;
* without friction the IMEX step is the RK32 step;
* the staged calls give the same step, and the step adjoint rejects IMEX.
"""
import numpy as np
import pytest

from helpers import build_oracle
from oracle import Mesh, Oracle, Params
from test_gpu_parity import (TOL_STEP, beach_crop, compare_states, cpu, gpu_from_oracle, hanging_case, n_r0_next,
                             rel, run_both, solver_for)
from workloads import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("crop", ["dam", "shore"])
def test_imex_beach_crop_steps(crop):
    say(f"case: 60 IMEX steps, beach crop {crop} 24x12, Manning 0.025")
    wl = beach_crop(116, 40) if crop == "dam" else beach_crop(200, 60, surge=(16200.0, 0.6))
    o, b = build_oracle(wl, rk="imex")
    s = solver_for(wl, o, b, rk="imex")
    s.set_state(*o.get_state())
    m0 = o.total_mass()
    d = run_both(o, s, 60)
    dg = s.diagnostics()
    say(f"  oracle dt {d['dt']:.6e} gpu dt {dg['dt']:.6e}; r0 {d['n_r0']} / {dg['n_r0_cells']}")
    compare_states(o, s, TOL_STEP, "60 steps")
    assert dg["n_r0_cells"] == n_r0_next(o)
    if crop == "shore":
        assert d["n_r0"] > 0
    assert dg["total_mass"] == pytest.approx(o.total_mass(), rel=1e-12)
    s.close()


@pytest.mark.parametrize("r,S", [(2, (16, 8)), (3, (16, 8, 5))])
def test_imex_hanging_tracer(r, S):
    say(f"case: 20 IMEX steps, hanging mesh + tracer + tide, Manning 0.03, r={r} S={S}")
    o, b = hanging_case(r, S)
    o.p.rk = "imex"
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    run_both(o, s, 20)
    compare_states(o, s, TOL_STEP, "20 steps")
    s.close()


def test_imex_stiff_uniform_friction():
    n, dt, nsteps = 0.5, 5.0, 8
    say(f"case: uniform flow, flat periodic bed, n={n}, dt={dt}, {nsteps} IMEX steps")
    m = Mesh.uniform(4, 4, 0.0, 0.0, 250.0, bc=("periodic",) * 4)
    o = Oracle(m, Params(r=1, S=(4,), rule="eq", rk="imex", eps=1e-3, h_lim=1e-3, adapt_degree=False))
    b = -np.ones(len(o.node_coords()))
    o.set_bathymetry(b)
    o.set_manning(np.full(m.K, n))
    sh = (m.K, o.np_)
    o.set_state(np.zeros(sh), np.ones(sh), np.zeros(sh))
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    for k in range(nsteps):
        o.step(dt)
        s.step(dt)
        s.sync()
        got = cpu(s.get_state()[1], m.K)
        ref = o.get_state()[1]
        e = np.abs(got - ref).max()
        say(f"  step {k + 1}: q oracle {ref.mean():+.6f} gpu {got.mean():+.6f} abs err {e:.2e}")
        assert e < 1e-12
    assert np.all(np.abs(o.get_state()[1]) <= 1.0)
    s.close()


def test_imex_without_friction_is_rk32():
    say("case: coastal_steps_16 (no friction), 30 steps, IMEX against RK32 on the GPU")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl, rk="rk32")
    s1 = solver_for(wl, o, b, rk="rk32")
    s2 = solver_for(wl, o, b, rk="imex")
    for s in (s1, s2):
        s.set_state(*o.get_state())
        for _ in range(30):
            s.step()
        s.sync()
    for f, name in enumerate(("eta", "qx", "qy")):
        e = rel(cpu(s2.get_state()[f], o.m.K), cpu(s1.get_state()[f], o.m.K))
        say(f"  {name} rel diff {e:.3e}")
        assert e < 1e-12
    s1.close()
    s2.close()


def test_imex_staged_calls_and_adjoint_rejection():
    say("case: IMEX step split into begin / rk_stage / end; sw_vjp_step rejects IMEX")
    wl = beach_crop(200, 60, nx=12, ny=8, surge=(16200.0, 0.6))
    o, b = build_oracle(wl, rk="imex")
    s1 = solver_for(wl, o, b, rk="imex")
    s2 = solver_for(wl, o, b, rk="imex")
    for s in (s1, s2):
        s.set_state(*o.get_state())
    for _ in range(5):
        s1.step()
        s2.step_begin()
        for l in range(2, 4):
            s2.rk_stage(l)
        s2.step_end()
    s1.sync()
    s2.sync()
    for f in range(3):
        assert np.array_equal(cpu(s1.get_state()[f], o.m.K), cpu(s2.get_state()[f], o.m.K))
    import torch
    stages = torch.zeros(3 * 3 * s1.n_dofs, dtype=torch.float64, device="cuda:0")
    s1.step_record(10.0, stages)
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(RuntimeError, match="IMEX"):
        s1.vjp_step(stages, 0.0, 10.0, z(3 * s1.n_dofs), z(s1.n_cells), z(s1.n_cells))
    s1.close()
    s2.close()


def test_imex_channel_parity():
    say("case: strong-friction channel (n = 1), N = 10, r = 1, IMEX at dt = 0.04 s (RK32 diverges at 0.02), 100 steps")
    from channel import channel_oracle, inflow
    o, b = channel_oracle(10, 1, "imex")
    s = gpu_from_oracle(o, b)
    s.set_boundary_state(inflow)
    s.set_state(*o.get_state())
    for _ in range(100):
        o.step(0.04)
        s.step(0.04)
    s.sync()
    got = [cpu(x, o.m.K) for x in s.get_state()[:3]]
    ref = o.get_state()
    qs = max(np.abs(ref[1]).max(), np.abs(ref[2]).max())
    errs = (rel(got[0], ref[0]), np.abs(got[1] - ref[1]).max() / qs, np.abs(got[2] - ref[2]).max() / qs)
    for name, e in zip(("zeta", "qx", "qy"), errs):
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_STEP
    s.close()


@pytest.mark.parametrize("r,Ns,rate", [(1, (20, 40), 1.6), (2, (10, 20), 1.8)])
def test_imex_channel_steady_state_converges(r, Ns, rate):
    """Sec. 4.3: the IMEX run from rest settles on a steady state whose surface
    converges to the ODE profile of eq:const_discharge as the mesh is refined
    (the paper's convergence study; 600 s of flow)."""
    from channel import channel_oracle, inflow, steady_profile
    xe, ze = steady_profile()
    errs = []
    for N in Ns:
        dt = 0.4 / N / r
        o, b = channel_oracle(N, r, "imex")
        s = gpu_from_oracle(o, b)
        s.set_boundary_state(inflow)
        s.set_state(*o.get_state())
        nst = int(round(600.0 / dt))
        s.run(nst - 1, dt)
        s.sync()
        z_prev = cpu(s.get_state()[0], N).copy()
        s.step(dt)
        s.sync()
        z = cpu(s.get_state()[0], N)
        d = o.dof_coords()
        e = float(np.sqrt(np.mean((z - np.interp(d[..., 0], xe, ze)) ** 2)))
        say(f"  r={r} N={N} dt={dt:.4f}: rms zeta error {e:.3e}, last-step change {np.abs(z - z_prev).max():.1e}")
        assert np.abs(z - z_prev).max() < 1e-8
        errs.append(e)
        s.close()
    got = np.log2(errs[0] / errs[1])
    say(f"  rate {got:.2f}")
    assert got > rate and errs[1] < 0.02
