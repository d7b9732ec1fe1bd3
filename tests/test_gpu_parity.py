"""GPU parity: the HIP library (through the C ABI) against the oracle, element
by element, on identical seeded inputs.

Tolerances (per field, relative to the oracle's max-norm): 1e-12 for one
residual evaluation, 1e-10 for the state after 100 steps.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

from helpers import build_oracle, mesh_from_desc
from oracle import Mesh, Oracle, Params
from workloads import quadtree_desc, uniform_mesh_desc, workload

pytestmark = pytest.mark.gpu

TOL_RHS = 1e-12
TOL_STEP = 1e-10


def say(*a):
    print(*a, flush=True)


def rel(g, r):
    g = np.asarray(g).ravel()
    r = np.asarray(r).ravel()
    scale = np.abs(r).max()
    return np.abs(g - r).max() / (scale if scale > 0 else 1.0)


def solver_for(wl, o, b, **over):
    from paper_2505_18743_amd import Solver
    params = dict(wl["params"])
    params.update(over)
    s = Solver(wl["mesh"], params, device="cuda:0")
    s.set_bathymetry(b)
    s.set_manning(wl["manning"] if "manning" in wl else np.zeros(o.m.K))
    return s


def cpu(t, K):
    return t.detach().cpu().numpy().reshape(K, -1)


def oracle_params(o):
    p = o.p
    return dict(r=p.r, S=p.S, rule=p.rule, rk=p.rk, g=p.g, eps=p.eps, h_lim=p.h_lim, eps0=p.eps0,
                newton_max=p.newton_max, cfl=p.cfl, cfl_mode=p.cfl_mode, tracer=p.tracer, tide=p.tide,
                adapt_degree=p.adapt_degree, tracer_diff=p.tracer_diff, tracer_strain=p.tracer_strain,
                tracer_decay=p.tracer_decay, quadrature=p.quadrature)


def mesh_dict(m):
    return dict(nx0=m.nx0, ny0=m.ny0, x0=m.x0, y0=m.y0, dx0=m.dx0, level=m.level, i=m.ii, j=m.jj, bc=m.bc)


def gpu_from_oracle(o, b, manning=None):
    from paper_2505_18743_amd import Solver
    s = Solver(mesh_dict(o.m), oracle_params(o), device="cuda:0")
    s.set_bathymetry(b)
    s.set_manning(manning if manning is not None else o.nman.numpy())
    return s


# ---------------------------------------------------------------------------

def test_coordinates_match_oracle():
    say("case: coordinates coastal_steps_16")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    assert np.abs(s.node_coords() - o.node_coords()).max() < 1e-12
    assert np.abs(s.dof_coords() - o.dof_coords().reshape(-1, 2)).max() < 1e-12


def test_apply_operator_coastal_steps():
    say("case: apply_operator coastal_steps_16")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    rng = np.random.default_rng(7)
    st = o.get_state()
    for trial in range(3):
        if trial > 0:      # random non-trivial states, including dry nodes
            st = [st[0] + rng.uniform(-0.3, 0.3, st[0].shape), rng.uniform(-1, 1, st[0].shape),
                  rng.uniform(-1, 1, st[0].shape), st[3]]
        F, Gx, Gy, R, dtb = o.apply_operator(st, 0.0)
        g = s.apply_operator(st[0], st[1], st[2], st[3], 0.0)
        s.sync()
        K = o.m.K
        for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy)):
            e = rel(cpu(gg, K), rr)
            say(f"  trial {trial} {name} rel err {e:.3e}")
            assert e < TOL_RHS, (trial, name, e)
        assert float(g[4].cpu()[0]) == pytest.approx(dtb, rel=1e-12)


def hanging_case(r=2, S=(16, 8), tracer=True, bc=("elev", "wall", "wall", "open")):
    def refine(L, cand):
        return [c for c in cand if (c[1] * 5 + c[2] * 3) % 4 == 0]
    d = quadtree_desc(6, 5, 0.0, 0.0, 400.0, refine, len(S) - 1, bc=bc)
    m = mesh_from_desc(d)
    p = Params(r=r, S=S, rule="eq", rk="ssp3", eps=0.05, h_lim=0.05, cfl=0.5, cfl_mode=1, tracer=tracer,
               tide=(0.3, 3000.0, 0.2, 0.25))
    o = Oracle(m, p)
    xy = o.node_coords()
    b = -3.0 + 4.5 * xy[:, 0] / 2400.0 + 0.6 * np.sin(xy[:, 1] / 150.0) * np.cos(xy[:, 0] / 90.0)
    b = np.where(np.abs(xy[:, 1] - 1010.0) < 60.0, b - 1.0, b)
    o.set_bathymetry(b)
    o.set_manning(np.full(m.K, 0.03))
    dof = o.dof_coords()
    eta = 0.4 * np.exp(-((dof[..., 0] - 700) ** 2 + (dof[..., 1] - 1000) ** 2) / 300.0 ** 2)
    c0 = np.exp(-((dof[..., 0] - 1200) ** 2 + (dof[..., 1] - 900) ** 2) / 400.0 ** 2)
    o.init_lake_at_rest(eta)
    o.state[3] = torch.as_tensor(c0)
    return o, b


@pytest.mark.parametrize("r,S", [(1, (8, 4)), (2, (16, 8)), (3, (16, 8, 5))])
def test_apply_operator_hanging_tracer(r, S):
    say(f"case: apply_operator hanging r={r} S={S}")
    o, b = hanging_case(r, S)
    assert any(f[4] >= 0 for f in o.m.faces)
    s = gpu_from_oracle(o, b)
    rng = np.random.default_rng(11)
    st = o.get_state()
    st = [st[0], rng.uniform(-0.5, 0.5, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape), st[3]]
    t = 700.0
    F, Gx, Gy, R, dtb = o.apply_operator(st, t)
    g = s.apply_operator(st[0], st[1], st[2], st[3], t)
    s.sync()
    K = o.m.K
    for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy), ("R", g[3], R)):
        e = rel(cpu(gg, K), rr)
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_RHS, (name, e)


def n_r0_next(o):
    """Cells at degree 0 for the next step: the library reports the degree
    decision it takes at the end of a step."""
    return int((o.adapted()[1] == 0).sum())


def compare_states(o, s, tol, label):
    """The library's step ends with the next step's start (degree decision and
    remap of cells going to degree 0), so its state is compared with the
    oracle's state after that same adaptation.

    The discharge, the depth integrals H_i and (with a tracer) the tracer
    masses int psi_i h c are compared in every cell.  The free surface and the
    concentration are compared in cells whose mean depth is at least h_lim:
    in a dry cell any zeta <= -max z_b is the same state, and in a nearly dry
    one zeta and c = (tracer mass) / Hbar change by |K| / (wet area) or
    1 / Hbar times the roundoff of their targets, so only the masses there
    are determined to roundoff."""
    K = o.m.K
    got = [cpu(t, K) for t in s.get_state()]
    ref = o.adapted_state()
    if not o.p.tracer:
        got[3] = ref[3] = np.zeros_like(ref[0])
    Hr, Cr, depth = o.conserved(ref)
    Hg, Cg, _ = o.conserved(got)
    wet = depth >= o.p.h_lim
    checks = [("qx", got[1], ref[1]), ("qy", got[2], ref[2]), ("H", Hg, Hr),
              ("eta (wet cells)", got[0][wet], ref[0][wet])]
    if o.p.tracer:
        checks += [("hc", Cg, Cr), ("c (wet cells)", got[3][wet], ref[3][wet])]
    for name, g, r_ in checks:
        e = rel(g, r_)
        say(f"  {label} {name} rel err {e:.3e}")
        assert e < tol, (label, name, e)


def run_both(o, s, nsteps, dt=None, check_every=None):
    dmax = 0
    for n in range(nsteps):
        d = o.step(dt)
        s.step(dt if dt else 0.0)
        if check_every and (n + 1) % check_every == 0:
            s.sync()
    s.sync()
    return d


def test_steps_coastal_steps_full_workload():
    """The 16x16 coastal workload for all its 100 SSP3 steps, CFL-controlled dt."""
    say("case: 100 steps coastal_steps_16")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    s.set_state(*o.get_state())
    m0 = o.total_mass()
    d = run_both(o, s, 100)
    dg = s.diagnostics()
    say(f"  oracle dt {d['dt']:.6e} gpu dt {dg['dt']:.6e}, r0 {d['n_r0']} / {dg['n_r0_cells']}")
    compare_states(o, s, TOL_STEP, "100 steps")
    assert dg["dt"] == pytest.approx(d["dt"], rel=1e-10)
    assert dg["t"] == pytest.approx(o.t, rel=1e-10)
    assert dg["total_mass"] == pytest.approx(m0, rel=1e-12)
    assert dg["n_r0_cells"] == n_r0_next(o)


def beach_crop(i0, j0, nx=24, ny=12, surge=None):
    wl = workload("beach_dambreak_256", window=(i0, j0, nx, ny))
    if surge is not None:         # a surge running up the dry beach
        x_front, level = surge
        wl["eta0"] = lambda x, y: np.where(np.asarray(x) < x_front, level, 0.0)
    return wl


@pytest.mark.parametrize("crop", ["dam", "shore"])
def test_steps_beach_dambreak_crop(crop):
    """Windows of the 256x256 case (same cell size, bed, r=2, 16x16 samples):
    the dam line, and the shoreline with a surge flooding dry cells."""
    say(f"case: 100 steps beach crop {crop} 24x12")
    wl = beach_crop(116, 40) if crop == "dam" else beach_crop(200, 60, surge=(16200.0, 0.6))
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    s.set_state(*o.get_state())
    d = run_both(o, s, 100)
    dg = s.diagnostics()
    say(f"  oracle newton {d['newton_it']} gpu {dg['max_newton_it']}; r0 {d['n_r0']} {dg['n_r0_cells']}")
    compare_states(o, s, TOL_STEP, "100 steps")
    assert dg["max_newton_it"] == d["newton_it"] and dg["n_r0_cells"] == n_r0_next(o)
    assert dg["n_fallback"] == d["n_fallback"]


@pytest.mark.parametrize("where", ["dam", "shore"])
def test_steps_beach_dambreak_crop_64(where):
    """64x64 windows of the 256x256 case (same cell size, bed, r=2, 16x16
    samples, Manning 0.025): across the dam line (all wet), and on the beach
    with a 0.6 m surge running up dry land (wet/dry, degree-0 cells).  100
    SSP3 steps at the CFL time step against the oracle."""
    say(f"case: 100 steps beach crop 64x64 ({where})")
    wl = beach_crop(100, 96, 64, 64) if where == "dam" else beach_crop(170, 96, 64, 64, surge=(15000.0, 0.6))
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    s.set_state(*o.get_state())
    for k in range(10):
        d = run_both(o, s, 10)
        say(f"  {10 * (k + 1)} steps, t = {o.t:.3f} s")
    dg = s.diagnostics()
    say(f"  oracle newton {d['newton_it']} gpu {dg['max_newton_it']}; r0 {d['n_r0']} {dg['n_r0_cells']}")
    compare_states(o, s, TOL_STEP, "100 steps")
    assert dg["t"] == pytest.approx(o.t, rel=1e-12)
    assert dg["n_r0_cells"] == n_r0_next(o) and (d["n_r0"] > 0) == (where == "shore")


@pytest.mark.parametrize("rk", ["ssp3", "rk32", "rk44", "fe"])
def test_steps_hanging_tracer_elev(rk):
    say(f"case: 20 steps hanging mesh + tracer + tide, {rk}")
    o, b = hanging_case(2, (16, 8))
    o.p.rk = rk
    if rk == "fe":
        o.p.cfl = 0.5
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    run_both(o, s, 20)
    compare_states(o, s, TOL_STEP, "20 steps")


@pytest.mark.parametrize("r", [1, 2, 3])
def test_wide_sample_rules_hanging_tracer(r):
    """20x20 samples on the coarse cells and 10x10 on the refined ones: the
    fast kernels run with 32 and 16 lanes per cell.  One residual evaluation
    and 10 SSP3 steps with tracer and tide against the oracle."""
    say(f"case: hanging mesh r={r} S=(20, 10)")
    o, b = hanging_case(r, (20, 10))
    s = gpu_from_oracle(o, b)
    st0 = o.get_state()
    K = o.m.K
    rng = np.random.default_rng(20 + r)
    st = [st0[0], rng.uniform(-0.5, 0.5, st0[0].shape), rng.uniform(-0.5, 0.5, st0[0].shape), st0[3]]
    F, Gx, Gy, R, dtb = o.apply_operator(st, 700.0)
    g = s.apply_operator(st[0], st[1], st[2], st[3], 700.0)
    s.sync()
    for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy), ("R", g[3], R)):
        e = rel(cpu(gg, K), rr)
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_RHS, (r, name, e)
    s.set_state(*st0)
    s.profile(True)
    s.kernel_time_reset()
    run_both(o, s, 10)
    launches = s.kernel_times()["element_stage"][1]
    s.profile(False)
    say(f"  fast stage kernel launches: {launches}")
    assert launches > 0
    compare_states(o, s, TOL_STEP, f"10 steps r={r}")
    s.close()


def test_stage_by_stage_matches_step():
    say("case: step split into begin / rk_stage / end")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s1 = solver_for(wl, o, b)
    s2 = solver_for(wl, o, b)
    st = o.get_state()
    s1.set_state(*st)
    s2.set_state(*st)
    for _ in range(3):
        s1.step()
        s2.step_begin()
        s2.rk_stage(2)
        s2.rk_stage(3)
        s2.step_end()
    s1.sync()
    s2.sync()
    for a, c in zip(s1.get_state(), s2.get_state()):
        assert torch.equal(a, c)


def test_lake_at_rest_init_matches_oracle():
    say("case: Definition 3.1 initialisation")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    dof = o.dof_coords()
    eta = wl["eta0"](dof[..., 0], dof[..., 1])
    s.init_lake_at_rest(eta)
    s.sync()
    K = o.m.K
    assert rel(cpu(s.get_state()[0], K), o.get_state()[0]) < 1e-15


@pytest.mark.parametrize("n,rk", [(1, "ssp3"), (3, "ssp3"), (5, "ssp3"), (1, "imex"), (5, "imex")])
def test_edge_single_and_ragged_meshes(n, rk):
    """1x1, 3x3, 5x5 meshes (cell counts not multiples of the cells per block), S=3 and S=5;
    with the IMEX pair under Manning friction too."""
    say(f"case: ragged {n}x{n}, {rk}")
    m = Mesh.uniform(n, n, 0.0, 0.0, 10.0)
    for (r, S) in ((1, 3), (2, 5)):
        p = Params(r=r, S=(S,), rule="gll", rk=rk, eps=1e-3, h_lim=1e-3, cfl=0.2)
        o = Oracle(m, p)
        xy = o.node_coords()
        b = -1.0 - 0.2 * np.sin(xy[:, 0] / 7.0) * np.cos(xy[:, 1] / 5.0)
        o.set_bathymetry(b)
        o.set_manning(np.full(m.K, 0.05 if rk == "imex" else 0.0))
        rng = np.random.default_rng(n + r)
        K, npn = m.K, (r + 1) ** 2
        st = [rng.uniform(-0.1, 0.1, (K, npn)), rng.uniform(-0.2, 0.2, (K, npn)), rng.uniform(-0.2, 0.2, (K, npn))]
        o.set_state(*st)
        s = gpu_from_oracle(o, b)
        F, Gx, Gy, R, dtb = o.apply_operator()
        g = s.apply_operator(*st, None, 0.0)
        s.sync()
        for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy)):
            assert rel(cpu(gg, K), rr) < TOL_RHS, (n, r, name)
        s.set_state(*st)
        run_both(o, s, 5)
        compare_states(o, s, TOL_STEP, f"{n}x{n} r={r}")


def full_beach(rk=None):
    wl = workload("beach_dambreak_256")
    if rk is not None:
        wl["params"] = dict(wl["params"], rk=rk)
    from paper_2505_18743_amd import Solver
    s = Solver(wl["mesh"], wl["params"], device="cuda:0")
    xy = s.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    s.set_bathymetry(b)
    s.set_manning(wl["manning"])
    dof = s.dof_coords()
    eta0 = wl["eta0"](dof[:, 0], dof[:, 1])
    s.init_lake_at_rest(eta0)
    return s, wl, b


def test_full_size_beach_sampled_residuals():
    """256x256, r=2, 16x16 samples, as the benchmark launches it: the residual of
    64 sampled cells against the oracle on the 3x3 patch around each."""
    say("case: full-size beach_dambreak_256 sampled residuals")
    s, wl, b = full_beach()
    s.run(10)
    assert beach_sampled_worst(s, wl, b) < TOL_RHS
    s.close()


def beach_sampled_worst(s, wl, b):
    st = [t.clone() for t in s.get_state()]
    g = s.apply_operator(st[0], st[1], st[2], None, 0.0)
    s.sync()
    n = 256
    npn = 9
    S = 16
    stn = [t.cpu().numpy().reshape(n, n, npn) for t in st[:3]]
    res = [t.cpu().numpy().reshape(n, n, npn) for t in g[:3]]
    bb = b.reshape(n, n, S * S)
    rng = np.random.default_rng(5)
    picks = [(int(rng.integers(1, n - 1)), int(rng.integers(1, n - 1))) for _ in range(56)]
    picks += [(j, 128) for j in (40, 90, 150, 200)] + [(70, 213), (71, 213), (140, 214), (141, 214)]
    scales = [max(np.abs(r_).max(), 1e-300) for r_ in res]   # full-field max-norms
    worst = 0.0
    for (j, i) in picks:
        m = Mesh.uniform(3, 3, (i - 1) * 78.125, (j - 1) * 78.125, 78.125)
        o = Oracle(m, Params(**{k: (tuple(v) if k in ("S", "tide") else v) for k, v in wl["params"].items()}))
        blk = bb[j - 1:j + 2, i - 1:i + 2].reshape(9, S * S)
        o.set_bathymetry(blk.ravel())
        o.set_manning(np.full(9, 0.025))
        patch = [a[j - 1:j + 2, i - 1:i + 2].reshape(9, npn) for a in stn]
        F, Gx, Gy, R, _ = o.apply_operator(patch + [np.zeros((9, npn))], 0.0)
        for gg, rr, scale in zip(res, (F, Gx, Gy), scales):
            worst = max(worst, np.abs(gg[j, i] - rr[4]).max() / scale)
    say(f"  worst sampled rel err {worst:.3e}")
    return worst


@pytest.mark.parametrize("rk,nsteps", [(None, 500), ("imex", 100)])
def test_full_size_beach_whole_run(rk, nsteps):
    """The benchmark's whole run (500 SSP3 steps of the 256x256 case; IMEX: 100
    steps): at every step the positivity bound holds (no cell target below
    roundoff: cells that are dry in exact arithmetic get targets like
    -1.6e-24 m^3 from cancellation) and every value is finite; the total mass
    (closed basin) is conserved to roundoff; at the end the operator still
    matches the oracle on sampled patches."""
    say(f"case: full-size beach_dambreak_256, {nsteps} steps, rk={rk or 'ssp3'}")
    s, wl, b = full_beach(rk)
    s.step()
    s.sync()
    m1 = s.diagnostics()["total_mass"]
    for k in range(nsteps - 1):
        s.step()
        d = s.diagnostics()
        assert d["min_target_mass"] >= -1e-12, (k, d)
        assert d["nonfinite"] == 0, (k, d)
    say(f"  mass {m1:.12e} -> {d['total_mass']:.12e}, t = {d['t']:.2f} s, cells of degree 0: {d['n_r0_cells']}")
    assert d["total_mass"] == pytest.approx(m1, rel=1e-12)
    assert beach_sampled_worst(s, wl, b) < TOL_RHS
    s.close()


@pytest.mark.parametrize("wpb,lanes,order", [(1, 2, 0), (2, 8, 1), (4, 4, 0), (1, 4, 0)])
def test_launch_shapes_give_the_same_step(wpb, lanes, order):
    say(f"case: launch shape wpb={wpb} lanes={lanes} order={order}, coastal_steps_16 + beach window, 10 steps")
    for name, kw in (("coastal_steps_16", {}), ("beach_dambreak_256", dict(window=(116, 40, 24, 12)))):
        wl = workload(name, **kw)
        o, b = build_oracle(wl)
        ref = solver_for(wl, o, b)
        alt = solver_for(wl, o, b)
        for s_ in (ref, alt):
            s_.set_state(*o.get_state())
        alt.set_workgroup(wpb, kernel=0)
        alt.set_workgroup(lanes, kernel=1)
        alt.set_workgroup(order, kernel=2)
        assert alt.get_workgroup(0, 0) == wpb and alt.get_workgroup(0, 1) == lanes
        assert alt.get_workgroup(0, 2) == order and ref.get_workgroup(0, 2) == 1
        ref.run(10)
        alt.run(10)
        ref.sync()
        alt.sync()
        a, r_ = ref.get_state(), alt.get_state()
        for f in range(3):
            e = rel(cpu(r_[f], o.m.K), cpu(a[f], o.m.K))
            say(f"  {name} field {f} rel diff {e:.3e}")
            # the element kernel's shape is exact; the face kernel's changes
            # the order of the face-node sums only (rounding, which wet/dry
            # fronts amplify over the steps: the after-steps bar applies)
            assert e < TOL_STEP, (name, f, e)
            if lanes == 4:
                assert torch.equal(a[f], r_[f]), (name, f)


def test_autotune_restores_the_state():
    say("case: sw_autotune on coastal_steps_16, then 5 steps vs 5 steps without tuning")
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    ref = solver_for(wl, o, b)
    tun = solver_for(wl, o, b)
    for s_ in (ref, tun):
        s_.set_state(*o.get_state())
        s_.run(3)
    choice = tun.autotune(steps=2)
    say(f"  chosen {choice}")
    assert choice["elem_waves_per_workgroup"] in (1, 2, 4) and choice["face_lanes"] in (2, 4, 8)
    ref.run(5)
    tun.run(5)
    ref.sync()
    tun.sync()
    dr, dt_ = ref.diagnostics(), tun.diagnostics()
    assert dr["t"] == pytest.approx(dt_["t"], rel=1e-13) and dr["step"] == dt_["step"]
    a, r_ = ref.get_state(), tun.get_state()
    for f in range(3):
        assert rel(cpu(r_[f], o.m.K), cpu(a[f], o.m.K)) < TOL_STEP


def test_full_size_tidal_quadtree_sampled_residuals():
    """The 2-level quadtree with about 120k leaves (r=3, 32/16/8 samples per
    level, tracer, tide on the west side), as built for the workload: the
    residual of sampled cells (every level, cells at hanging faces and at the
    tidal boundary) against the oracle on the 3x3 window of coarse cells around
    each, with the library's own sample values."""
    say("case: full-size tidal_quadtree_r3 sampled residuals")
    from paper_2505_18743_amd import Solver
    wl = workload("tidal_quadtree_r3")
    d = wl["mesh"]
    s = Solver(d, wl["params"], device="cuda:0")
    xy = s.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    del xy
    s.set_bathymetry(b)
    s.set_manning(wl["manning"])
    dof = s.dof_coords()
    s.init_lake_at_rest(wl["eta0"](dof[:, 0], dof[:, 1]))
    st = s.get_state()
    L = d["nx0"] * d["dx0"]
    x, y = dof[:, 0], dof[:, 1]
    eta = st[0].cpu().numpy() + 0.4 * np.exp(-((x - 0.3 * L) ** 2 + (y - 0.6 * L) ** 2) / (0.1 * L) ** 2)
    qx = 0.3 * np.sin(x / 3000.0) * np.cos(y / 2500.0)
    qy = 0.2 * np.cos(x / 2000.0 + 0.5) * np.sin(y / 3500.0)
    c = wl["tracer0"](x, y)
    t = 3000.0
    worst, nh, nw = quadtree_sampled_worst(s, wl, b, [eta, qx, qy, c], t)
    assert nh == 8 and nw == 4
    assert worst < TOL_RHS
    s.close()


def quadtree_sampled_worst(s, wl, b, state, t):
    """Worst sampled residual error of the quadtree context s at `state`
    against the oracle on 3x3 coarse-cell windows (every level, cells at
    hanging faces, cells on the tidal side)."""
    d = wl["mesh"]
    eta, qx, qy, c = state
    g = s.apply_operator(eta, qx, qy, c, t)
    s.sync()
    K, NP = s.n_cells, s.np_
    res = [r_.cpu().numpy().reshape(K, NP) for r_ in g[:4]]
    state = [np.asarray(v).reshape(K, NP) for v in (eta, qx, qy, c)]
    scales = [max(np.abs(r_).max(), 1e-300) for r_ in res]
    # context order: by level, then the description's order
    member, local = s.cell_map()
    lev, ci, cj = d["level"][local], d["i"][local], d["j"][local]
    S = wl["params"]["S"]
    nodes_per = np.array([S[l] ** 2 for l in lev])
    noff = np.concatenate([[0], np.cumsum(nodes_per)])
    key = {(int(lev[k]), int(ci[k]), int(cj[k])): k for k in range(K)}
    coarse = np.stack([ci >> lev, cj >> lev], 1)
    # picks: every level, cells next to a coarser or finer leaf, west boundary cells
    rng = np.random.default_rng(17)
    picks = []
    for lv in range(3):
        ks = np.nonzero(lev == lv)[0]
        picks += list(rng.choice(ks, 6, replace=False))
    hang = [k for k in rng.permutation(K)[:4000]
            if any((int(lev[k]) - 1, int(ci[k] + di) >> 1, int(cj[k] + dj) >> 1) in key
                   for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)))][:8]
    west = [k for k in rng.permutation(K)[:20000] if ci[k] == 0][:4]
    picks += hang + west
    pkw = {k: v for k, v in wl["params"].items()}
    params = Params(**{k: (tuple(v) if k in ("S", "tide") else v) for k, v in pkw.items()})
    worst = 0.0
    for k in picks:
        cx, cy = coarse[k]
        x0, x1 = max(cx - 1, 0), min(cx + 1, d["nx0"] - 1)
        y0, y1 = max(cy - 1, 0), min(cy + 1, d["ny0"] - 1)
        sel = np.nonzero((coarse[:, 0] >= x0) & (coarse[:, 0] <= x1) & (coarse[:, 1] >= y0) & (coarse[:, 1] <= y1))[0]
        wlev = lev[sel]
        m = Mesh(x1 - x0 + 1, y1 - y0 + 1, d["x0"] + x0 * d["dx0"], d["y0"] + y0 * d["dx0"], d["dx0"], wlev,
                 ci[sel] - (x0 << wlev), cj[sel] - (y0 << wlev),
                 ("elev" if x0 == 0 else "wall", "wall", "wall", "wall"))
        o = Oracle(m, params)
        o.set_bathymetry(np.concatenate([b[noff[q]:noff[q + 1]] for q in sel]))
        o.set_manning(np.full(len(sel), 0.025))
        F, Gx, Gy, R, _ = o.apply_operator([v[sel] for v in state], t)
        w = int(np.nonzero(sel == k)[0][0])
        for gg, rr, scale in zip(res, (F, Gx, Gy, R), scales):
            worst = max(worst, np.abs(gg[k] - rr[w]).max() / scale)
    say(f"  {len(picks)} sampled cells ({len(hang)} at hanging faces, {len(west)} on the tidal side), "
        f"worst rel err {worst:.3e}")
    return worst, len(hang), len(west)


def test_full_size_tidal_quadtree_whole_run():
    """The quadtree workload's whole run (1000 coupled steps with tracer and
    tide): finite values and positivity to roundoff along the run, then the
    operator at the final state against the oracle on sampled windows."""
    say("case: full-size tidal_quadtree_r3, 1000 steps")
    from paper_2505_18743_amd import Solver
    wl = workload("tidal_quadtree_r3")
    d = wl["mesh"]
    s = Solver(d, wl["params"], device="cuda:0")
    xy = s.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    del xy
    s.set_bathymetry(b)
    s.set_manning(wl["manning"])
    dof = s.dof_coords()
    s.init_lake_at_rest(wl["eta0"](dof[:, 0], dof[:, 1]))
    st = s.get_state()
    s.set_state(st[0], st[1], st[2], wl["tracer0"](dof[:, 0], dof[:, 1]))
    for k in range(20):
        s.run(50)
        dg = s.diagnostics()
        assert dg["nonfinite"] == 0 and dg["min_target_mass"] >= -1e-12, (k, dg)
    say(f"  t = {dg['t']:.1f} s after {dg['step']} steps, cells of degree 0: {dg['n_r0_cells']}")
    # after 1000 steps of a slow tide the basin is still near rest, where the
    # residuals are roundoff of the balanced hydrostatic terms; the operator
    # check adds the same surface hump and discharge field as the sampled
    # test above to the final surface, so every residual has a scale of its own
    st = [x.detach().cpu().numpy() for x in s.get_state()]
    L = d["nx0"] * d["dx0"]
    x, y = dof[:, 0], dof[:, 1]
    st[0] = st[0] + 0.4 * np.exp(-((x - 0.3 * L) ** 2 + (y - 0.6 * L) ** 2) / (0.1 * L) ** 2)
    st[1] = st[1] + 0.3 * np.sin(x / 3000.0) * np.cos(y / 2500.0)
    st[2] = st[2] + 0.2 * np.cos(x / 2000.0 + 0.5) * np.sin(y / 3500.0)
    worst, nh, nw = quadtree_sampled_worst(s, wl, b, st, dg["t"])
    assert worst < TOL_RHS
    s.close()


@pytest.mark.parametrize("rk", ["ssp3", "imex"])
def test_all_dry_domain(rk):
    """A domain dry everywhere, 5 fixed-dt steps with tracer and friction: the
    surface the dry lift and the scalar solve leave matches the oracle; depth,
    discharge and tracer stay at rest to roundoff; nothing becomes non-finite."""
    say(f"case: all-dry 4x3 mesh, r=2, {rk}")
    from test_oracle_properties import all_dry_case
    o, b = all_dry_case(rk)
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    for _ in range(5):
        o.step(1.0)
        s.step(1.0)
    s.sync()
    K = o.m.K
    got = [cpu(x, K) for x in s.get_state()]
    ref = o.get_state()
    e = rel(got[0], ref[0])
    say(f"  zeta rel err {e:.3e}, max |q| {max(np.abs(got[1]).max(), np.abs(got[2]).max()):.2e}, "
        f"max |c - 0.7| {np.abs(got[3] - 0.7).max():.2e}")
    assert e < TOL_STEP
    assert all(np.all(np.isfinite(v)) for v in got)
    assert np.abs(got[1]).max() < 1e-25 and np.abs(got[2]).max() < 1e-25
    assert np.abs(got[3] - 0.7).max() < 1e-14
    dg = s.diagnostics()
    assert dg["n_r0_cells"] == K and abs(dg["total_mass"]) < 1e-13 and dg["nonfinite"] == 0
    s.close()


def tidal_quadtree_window(x0, y0, n, hump=0.0):
    """A window of n x n coarse cells of the tidal quadtree workload (its
    leaves there, its bed, its rule r = 3 with 32/16/8 samples per level,
    its time step, tide and Manning 0.025); the west side is tidal when the
    window touches it, the other sides are walls.  The surface carries a
    Gaussian hump of the given height in the window (Def. 3.1 dry rule) and
    the tracer a Gaussian."""
    wl = workload("tidal_quadtree_r3")
    d = wl["mesh"]
    lev, ci, cj = d["level"], d["i"], d["j"]
    sel = ((ci >> lev) >= x0) & ((ci >> lev) < x0 + n) & ((cj >> lev) >= y0) & ((cj >> lev) < y0 + n)
    L = lev[sel]
    dx0 = d["dx0"]
    m = Mesh(n, n, d["x0"] + x0 * dx0, d["y0"] + y0 * dx0, dx0, L, ci[sel] - (x0 << L), cj[sel] - (y0 << L),
             ("elev" if x0 == 0 else "wall", "wall", "wall", "wall"))
    pd = dict(wl["params"])
    o = Oracle(m, Params(**{k: (tuple(v) if k in ("S", "tide") else v) for k, v in pd.items()}))
    xy = o.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    o.set_bathymetry(b)
    o.set_manning(np.full(m.K, 0.025))
    dof = o.dof_coords()
    xc, yc = m.x0 + 0.5 * n * dx0, m.y0 + 0.5 * n * dx0
    c0 = np.exp(-((dof[..., 0] - xc) ** 2 + (dof[..., 1] - yc) ** 2) / (2.0 * 300.0 ** 2))
    eta = hump * np.exp(-((dof[..., 0] - xc) ** 2 + (dof[..., 1] - yc) ** 2) / (2.0 * 200.0 ** 2))
    o.init_lake_at_rest(eta)
    o.state[3] = torch.as_tensor(c0)
    return o, b


@pytest.mark.parametrize("where", ["tide", "islands"])
def test_steps_tidal_quadtree_window_c3_rule(where):
    """The quadtree workload's own discretisation on 6 x 6 coarse-cell
    windows (three levels with 32, 16 and 8 samples per direction, so the
    fast kernels run 32, 16 and 8 lanes per cell), with tracer and Manning
    friction: at the tidal side with a 0.3 m hump, and around islands with a
    1 m hump flooding them (wet/dry cells, degree-0 cells).  100 SSP3 steps at
    the workload's CFL time step against the oracle, every field."""
    say(f"case: 100 steps tidal quadtree window 6x6 ({where}), r=3, S=(32,16,8)")
    o, b = tidal_quadtree_window(0, 40, 6, hump=0.3) if where == "tide" else \
        tidal_quadtree_window(96, 72, 6, hump=1.0)
    assert sorted(set(o.m.level.tolist())) == [0, 1, 2] and any(f[4] >= 0 for f in o.m.faces)
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    for k in range(10):
        d = run_both(o, s, 10)
        say(f"  {10 * (k + 1)} steps, t = {o.t:.3f} s")
    dg = s.diagnostics()
    say(f"  oracle newton {d['newton_it']} gpu {dg['max_newton_it']}; r0 {d['n_r0']} {dg['n_r0_cells']}")
    compare_states(o, s, TOL_STEP, "100 steps")
    assert dg["t"] == pytest.approx(o.t, rel=1e-12)
    assert dg["n_r0_cells"] == n_r0_next(o) and dg["max_newton_it"] == d["newton_it"]
    s.close()


def test_set_tide_equals_the_created_tide():
    """sw_set_tide on a context made without a tide gives the steps of a
    context made with it, bit for bit (hanging mesh, elevation side, tracer)."""
    say("case: sw_set_tide vs the tide of sw_params, hanging mesh, 10 steps")
    o, b = hanging_case(2, (16, 8))
    s1 = gpu_from_oracle(o, b)
    p0 = oracle_params(o)
    p0["tide"] = (0.0, 1.0, 0.0, 0.0)
    from paper_2505_18743_amd import Solver
    s2 = Solver(mesh_dict(o.m), p0, device="cuda:0")
    s2.set_bathymetry(b)
    s2.set_manning(o.nman.numpy())
    s2.set_tide(*o.p.tide)
    with pytest.raises(RuntimeError, match="period"):
        s2.set_tide(0.3, 0.0)
    st = o.get_state()
    for s in (s1, s2):
        s.set_state(*st)
        for _ in range(10):
            s.step()
        s.sync()
    for f in range(4):
        assert torch.equal(s1.get_state()[f], s2.get_state()[f]), f
    s1.close()
    s2.close()
