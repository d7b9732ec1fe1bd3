"""GPU: dynamic h-adaptivity (Sec. 3.3 criteria; Sec. 3.4 conservative remap,
eq:cons-remap, and Q^n, eq:mass-loss) through the C ABI against the oracle.

* The indicators (vorticity, tracer gradient) on a two-level wet/dry mesh,
  with the sample rule and with the paper's quadrature: 1e-12.
* Remeshes of that case between steps (bathymetry from a rough raster,
  per-cell Manning coefficients and bed offsets, tracer, tide): the new
  leaves and the refine / merge counts equal the oracle's exactly; eta_max,
  the masses before and after and Q^n to 1e-12; the transferred state to
  1e-12; the steps after each remesh to 1e-10.
* The travelling vortex of Sec. 4.4 with AMR (RK32, r = 1, n_max = 2, the
  paper's thresholds, remesh every 5 steps): 12 steps with two remeshes
  against the oracle (1e-10); the whole run on the GPU, whose L2 errors equal
  the static finest mesh's within 0.5 % with less than half its degrees of
  freedom, at n_max = 2 and 3 (Table 7's AMR columns).
* Argument checks.
"""
import math

import numpy as np
import pytest
import torch

from exact import G, Vortex
from helpers import mesh_from_desc
from oracle import Mesh, Oracle, Params
from oracle.amr import TRACER_GRAD, VORTICITY, indicator, remesh, sample_raster
from test_gpu_parity import TOL_RHS, TOL_STEP, compare_states, cpu, mesh_dict, oracle_params, rel
from test_gpu_paper_quadrature import l2_errors_state
from test_oracle_paper_quadrature import l2_project
from workloads import quadtree_desc

pytestmark = pytest.mark.gpu

TOL_XFER = 1e-12


def say(*a):
    print(*a, flush=True)


def raster(seed=3):
    """A rough bed over [0, 2400] x [0, 2000]: a slope, ripples, a trench and noise."""
    rng = np.random.default_rng(seed)
    x = np.arange(0.0, 2410.0, 20.0)
    y = np.arange(0.0, 2010.0, 20.0)
    X, Y = np.meshgrid(x, y)
    b = -3.0 + 4.5 * X / 2400.0 + 0.6 * np.sin(Y / 150.0) * np.cos(X / 90.0)
    b = np.where(np.abs(Y - 1010.0) < 60.0, b - 1.0, b) + 0.05 * rng.normal(size=b.shape)
    return dict(x0=0.0, y0=0.0, dx=20.0, dy=20.0, b=b)


def coastal_amr(r=2, quadrature="subgrid", rk="ssp3"):
    def refine(L, cand):
        return [c for c in cand if (c[1] * 5 + c[2] * 3) % 4 == 0]
    d = quadtree_desc(6, 5, 0.0, 0.0, 400.0, refine, 1, bc=("elev", "wall", "wall", "open"))
    m = mesh_from_desc(d)
    S = (r + 2,) * 3 if quadrature == "paper" else (8, 8, 8)
    p = Params(r=r, S=S, rule="gll" if quadrature == "paper" else "eq", rk=rk, eps=0.05, h_lim=0.05, cfl=0.3,
               cfl_mode=1, tracer=True, tide=(0.3, 3000.0, 0.2, 0.25), quadrature=quadrature)
    o = Oracle(m, p)
    grid = raster()
    o.set_bathymetry(sample_raster(grid, o.node_coords()))
    o.set_manning(0.02 + 0.01 * np.sin(np.arange(m.K)))
    o.set_bed_offset(0.05 * np.cos(np.arange(m.K) / 3.0))
    dof = o.dof_coords()
    eta = 0.4 * np.exp(-((dof[..., 0] - 700) ** 2 + (dof[..., 1] - 1000) ** 2) / 300.0 ** 2)
    c0 = np.exp(-((dof[..., 0] - 1200) ** 2 + (dof[..., 1] - 900) ** 2) / 400.0 ** 2)
    o.init_lake_at_rest(eta)
    o.state[3] = torch.as_tensor(c0)
    return o, grid


def gpu_amr(o, grid):
    from paper_2505_18743_amd import Solver
    s = Solver(mesh_dict(o.m), oracle_params(o), device="cuda:0")
    s.set_bed_grid(grid)
    s.set_manning(o.nman.numpy())
    s.set_bed_offset(o.dbed.numpy())
    s.set_state(*o.get_state())
    return s


def same_mesh(o, s):
    lev, ii, jj = s.cells()
    return (np.array_equal(lev, o.m.level) and np.array_equal(ii, o.m.ii) and np.array_equal(jj, o.m.jj))


@pytest.mark.parametrize("quadrature", ["subgrid", "paper"])
def test_indicator_parity(quadrature):
    say(f"case: AMR indicators, two levels, wet/dry, tracer, {quadrature} quadrature")
    o, grid = coastal_amr(quadrature=quadrature)
    s = gpu_amr(o, grid)
    assert np.abs(s.node_coords() - o.node_coords()).max() < 1e-9
    for _ in range(3):
        o.step()
        s.step()
    for kind, name in ((VORTICITY, "vorticity"), (TRACER_GRAD, "tracer_grad")):
        ref = indicator(o, kind)
        got = s.amr_indicator(name).cpu().numpy()
        e = rel(got, ref)
        say(f"  {name}: max {ref.max():.4e}, rel err {e:.3e}")
        assert ref.max() > 0 and e < TOL_RHS, (name, e)
    s.close()


def fragile(o, state):
    """sum of w |z_b| over the sample nodes whose depth zeta + z_b is within 1e-9 of zero"""
    tot = 0.0
    for lv in o.levels:
        if len(lv.idx) == 0:
            continue
        zb = o.zb_eff(lv)
        sdep = torch.as_tensor(np.asarray(state[0])[lv.idx.numpy()]) @ lv.Bv.T + zb
        tot += float((lv.W * zb.abs())[sdep.abs() < 1e-9].sum())
    return tot


def check_remesh(o, s, grid, kind, name, tr, tc, nmax, label):
    n, rel_, st = remesh(o, grid, kind, tr, tc, nmax)
    gs = s.remesh(name, tr, tc, nmax)
    say(f"  {label}: {st['n_cells_old']} -> {st['n_cells_new']} cells, refined {st['n_refined']}, "
        f"merged {st['n_coarsened']}, Q^n {st['q_bathy']:.4e}, mass {st['mass_old']:.6e} -> {st['mass_new']:.6e}")
    for k in ("n_cells_old", "n_cells_new", "n_refined", "n_coarsened"):
        assert gs[k] == st[k], (label, k, gs[k], st[k])
    for k in ("eta_max", "mass_old", "mass_new"):
        assert abs(gs[k] - st[k]) <= 1e-12 * abs(st[k]), (label, k, gs[k], st[k])
    # Q^n weighs z_b by the land-sea mask, which a node where the surface meets
    # the bed (depth below 1e-9, e.g. a dry cell's deepest node) may take
    # either way under roundoff: such nodes bound the difference
    tol = fragile(o, o.adapted_state()) + fragile(n, n.get_state()) + 1e-12 * st["mass_old"]
    assert abs(gs["q_bathy"] - st["q_bathy"]) <= tol, (label, gs["q_bathy"], st["q_bathy"], tol)
    assert same_mesh(n, s), label
    assert np.abs(s.node_coords() - n.node_coords()).max() < 1e-9
    got = [cpu(t, n.m.K) for t in s.get_state()]
    for f, fname in enumerate(("zeta", "qx", "qy", "c")):
        e = rel(got[f], n.get_state()[f])
        assert e < TOL_XFER, (label, fname, e)
    return n, st


@pytest.mark.parametrize("quadrature,rk", [("subgrid", "ssp3"), ("paper", "ssp3"), ("subgrid", "imex")])
def test_remesh_and_steps_parity(quadrature, rk):
    say(f"case: remesh between steps, two to three levels, wet/dry, raster bed, {quadrature} quadrature, {rk}")
    o, grid = coastal_amr(quadrature=quadrature, rk=rk)
    s = gpu_amr(o, grid)
    for _ in range(5):
        o.step()
        s.step()
    o, st = check_remesh(o, s, grid, VORTICITY, "vorticity", 0.3, 0.05, 3, "vorticity remesh")
    assert st["n_refined"] > 0 and st["n_coarsened"] > 0
    for _ in range(5):
        o.step()
        s.step()
    s.sync()
    assert s.diagnostics()["t"] == pytest.approx(o.t, rel=1e-12)
    compare_states(o, s, TOL_STEP, "5 steps after the first remesh")
    o, st = check_remesh(o, s, grid, TRACER_GRAD, "tracer_grad", 0.2, 0.02, 3, "tracer remesh")
    assert st["n_refined"] + st["n_coarsened"] > 0
    for _ in range(5):
        o.step()
        s.step()
    s.sync()
    compare_states(o, s, TOL_STEP, "5 steps after the second remesh")
    s.close()


def test_remesh_without_change_keeps_the_context():
    say("case: remesh with thresholds that select nothing")
    o, grid = coastal_amr()
    s = gpu_amr(o, grid)
    s.step()
    before = [cpu(t, o.m.K) for t in s.get_state()]
    st = s.remesh("vorticity", 2.0, 0.0, 3)
    assert st["n_refined"] == 0 and st["n_coarsened"] == 0 and st["n_cells_new"] == o.m.K
    after = [cpu(t, o.m.K) for t in s.get_state()]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    s.close()


def vortex_case(N, nmax, r=1, rk="rk32", static=False):
    from paper_2505_18743_amd import Solver
    Nm = N * 2 ** (nmax - 1) if static else N
    m = Mesh.uniform(2 * Nm, Nm, 0.0, 0.0, 1.0 / Nm, bc=("state", "open", "wall", "wall"))
    p = Params(r=r, S=(r + 2,) * (1 if static else nmax), rule="gll", rk=rk, eps=1e-3, h_lim=0.0,
               adapt_degree=False, quadrature="paper")
    o = Oracle(m, p)
    grid = dict(x0=-1.0, y0=-1.0, dx=4.0, dy=3.0, b=np.zeros((2, 2)))
    o.set_bathymetry(sample_raster(grid, o.node_coords()))
    s = Solver(mesh_dict(m), oracle_params(o), device="cuda:0")
    s.set_bed_grid(grid)
    s.set_manning(np.zeros(m.K))
    return o, s, grid


def exact_fn(v, t):
    def fn(x, y):
        h, u, w = v.fields(x, y, t)
        return h, h * u, h * w, np.zeros_like(x)
    return fn


def run_vortex_gpu(N, nmax, static, T, cfl=0.2, r=1, rk="rk32", oracle_steps=0):
    v = Vortex()
    o, s, grid = vortex_case(N, nmax, r, rk, static)
    init = l2_project(o.m, r, lambda x, y: exact_fn(v, 0.0)(x, y)[:3])
    o.set_state(*init)
    s.set_state(*init)
    if not static:   # the initial mesh adapted to the initial state
        for _ in range(nmax - 1):
            if oracle_steps:
                o, _, _ = remesh(o, grid, VORTICITY, 1e-4, 5e-5, nmax)
            s.remesh("vorticity", 1e-4, 5e-5, nmax)
            lev, ii, jj = s.cells()
            mm = Mesh(o.m.nx0, o.m.ny0, 0.0, 0.0, o.m.dx0, lev, ii, jj, o.m.bc)
            init = l2_project(mm, r, lambda x, y: exact_fn(v, 0.0)(x, y)[:3])
            if oracle_steps:
                assert same_mesh(o, s)
                o.set_state(*init)
            s.set_state(*init)
    Nf = N * 2 ** (nmax - 1)
    n = int(math.ceil(T / (cfl / Nf / (6.9 + math.sqrt(G)))))
    dt = T / n
    for k in range(n):
        if not static and k > 0 and k % 5 == 0:
            st = s.remesh("vorticity", 1e-4, 5e-5, nmax)
            assert abs(st["mass_new"] - st["mass_old"]) < 1e-12 * st["mass_old"]
            if k < oracle_steps:
                o, _, _ = remesh(o, grid, VORTICITY, 1e-4, 5e-5, nmax)
                assert same_mesh(o, s)
        s.set_boundary_state(exact_fn(v, k * dt))
        s.step(dt)
        if k < oracle_steps:
            o.set_boundary_state(exact_fn(v, k * dt))
            o.step(dt)
            if k == oracle_steps - 1:
                s.sync()
                for f, name in enumerate(("zeta", "qx", "qy")):
                    e = rel(cpu(s.get_state()[f], o.m.K), o.get_state()[f])
                    say(f"  {oracle_steps} steps vs the oracle: {name} rel err {e:.3e}")
                    assert e < TOL_STEP, (name, e)
    s.sync()
    lev, ii, jj = s.cells()
    m = Mesh(2 * N if not static else 2 * Nf, N if not static else Nf, 0.0, 0.0,
             1.0 / (N if not static else Nf), lev, ii, jj, ("state", "open", "wall", "wall"))
    st = [cpu(x, m.K) for x in s.get_state()[:3]]
    ez, eq = l2_errors_state(st, m, r, v, T)
    dofs = m.K * (r + 1) ** 2 * 3
    s.close()
    return ez, eq, dofs


def test_vortex_amr_against_the_oracle():
    say("case: vortex with AMR, RK32 r=1 n_max=2, 12 steps with two remeshes against the oracle")
    run_vortex_gpu(20, 2, False, T=1.0 / 6.0, oracle_steps=12)


@pytest.mark.parametrize("nmax", [2, 3])
def test_vortex_amr_matches_static(nmax):
    say(f"case: vortex AMR vs static finest mesh, RK32 r=1 n_max={nmax}, T=1/6 on the GPU")
    T = 1.0 / 6.0
    sz, sq, sd = run_vortex_gpu(20, nmax, True, T)
    az, aq, ad = run_vortex_gpu(20, nmax, False, T)
    say(f"  static {sd} dofs: {sz:.4e} {sq:.4e}; AMR {ad} dofs: {az:.4e} {aq:.4e}")
    assert abs(az / sz - 1.0) < 5e-3 and abs(aq / sq - 1.0) < 5e-3
    assert ad < 0.5 * sd


def test_boundary_data_carry_over():
    say("case: vortex AMR, the inflow side's data carry over a remesh that leaves its faces alone")
    from paper_2505_18743_amd import Solver
    v = Vortex()
    out = []
    for reset in (False, True):
        o, s, grid = vortex_case(20, 2)
        init = l2_project(o.m, 1, lambda x, y: exact_fn(v, 0.0)(x, y)[:3])
        s.set_state(*init)
        s.set_boundary_state(exact_fn(v, 0.0))
        for _ in range(3):
            s.step(1e-4)
        st = s.remesh("vorticity", 1e-4, 5e-5, 2)
        assert st["n_refined"] > 0 and st["boundary_data_kept"] == 1
        if reset:
            s.set_boundary_state(exact_fn(v, 0.0))
        for _ in range(3):
            s.step(1e-4)
        s.sync()
        out.append([cpu(x, s.n_cells) for x in s.get_state()[:3]])
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_amr_argument_checks():
    from paper_2505_18743_amd import Solver
    say("case: AMR argument checks")
    m = Mesh.uniform(4, 3, 0.0, 0.0, 1.0)
    p = dict(r=1, S=(4, 4), rule="eq", rk="ssp3")
    s = Solver(mesh_dict(m), p, device="cuda:0")
    s.set_bathymetry(np.full(s.n_vol, -1.0))
    s.set_manning(np.zeros(m.K))
    s.set_state(np.zeros((m.K, 4)), np.zeros((m.K, 4)), np.zeros((m.K, 4)))
    with pytest.raises(RuntimeError, match="raster"):
        s.remesh("vorticity", 0.5, 0.1, 2)
    s.set_bed_grid(dict(x0=0.0, y0=0.0, dx=1.0, dy=1.0, b=np.full((4, 5), -1.0)))
    with pytest.raises(RuntimeError, match="n_max"):
        s.remesh("vorticity", 0.5, 0.1, 3)
    with pytest.raises(RuntimeError, match="tracer"):
        s.remesh("tracer_grad", 0.5, 0.1, 2)
    s.close()
    b = Solver([mesh_dict(m), mesh_dict(m)], [p, p], device="cuda:0")
    b.set_bathymetry(np.full(b.n_vol, -1.0))
    with pytest.raises(RuntimeError, match="single-member"):
        b.remesh("vorticity", 0.5, 0.1, 2)
    b.close()
