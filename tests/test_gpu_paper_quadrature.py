"""GPU: the library with the quadrature of Table 1 (SW_QUAD_PAPER: volume
terms on Gauss-Legendre (floor(3r/2)+1)^2 nodes with bathymetry samples of
their own, faces, wet/dry rule and continuity / tracer mass on GLL (r+2)^2,
the exact discharge mass) against the oracle in the same mode, and the
travelling vortex of Sec. 4.4 against the errors Table 7 prints.

* node coordinates (sample nodes, then volume-rule nodes) equal the oracle's;
* one residual evaluation on a two-level mesh with wet/dry cells, Manning
  friction and a tracer with diffusion and decay, r = 1..3: 1e-12;
* steps of that case (SSP3 and IMEX, degree adaptation on), compared as the
  other step tests: 1e-10;
* the vortex at N = 20 with the exact inflow state, 10 steps against the
  oracle (1e-10), and the whole run to T = 1/6 on the GPU alone, whose L2
  errors must match Table 7 as the oracle's do (3 %, 3 %, 0.5 %);
* the argument checks (GLL with S = r + 2 only; no adjoint).
"""
import math

import numpy as np
import pytest
import torch

from exact import Vortex
from helpers import mesh_from_desc
from oracle import Mesh, Oracle, Params, gl_rule, tensor_basis
from test_gpu_parity import TOL_RHS, TOL_STEP, compare_states, cpu, gpu_from_oracle, mesh_dict, rel
from test_oracle_paper_quadrature import l2_project, table7
from workloads import quadtree_desc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def coastal_paper(r, rk="ssp3", tracer=True):
    """Two-level mesh over a sloping beach with a bump and a trench, a Gaussian
    hump of water, Manning friction and a tracer with diffusion and decay."""
    def refine(L, cand):
        return [c for c in cand if (c[1] * 5 + c[2] * 3) % 4 == 0]
    d = quadtree_desc(6, 5, 0.0, 0.0, 400.0, refine, 1, bc=("elev", "wall", "wall", "open"))
    m = mesh_from_desc(d)
    p = Params(r=r, S=(r + 2, r + 2), rule="gll", rk=rk, eps=0.05, h_lim=0.05, cfl=0.3, cfl_mode=1,
               tracer=tracer, tide=(0.3, 3000.0, 0.2, 0.25), tracer_diff=0.33, tracer_strain=0.004,
               tracer_decay=2e-4, quadrature="paper")
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


@pytest.mark.parametrize("r", [1, 2, 3])
def test_node_coords_paper(r):
    say(f"case: node coordinates, paper quadrature r={r}")
    o, b = coastal_paper(r)
    nv = (3 * r) // 2 + 1
    assert len(b) == o.m.K * ((r + 2) ** 2 + nv * nv)
    s = gpu_from_oracle(o, b)
    assert np.abs(s.node_coords() - o.node_coords()).max() < 1e-9
    s.close()


@pytest.mark.parametrize("r", [1, 2, 3])
def test_apply_operator_paper(r):
    say(f"case: apply_operator, paper quadrature, two levels, wet/dry, tracer sources r={r}")
    o, b = coastal_paper(r)
    s = gpu_from_oracle(o, b)
    rng = np.random.default_rng(5 + r)
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
    assert float(g[4].cpu()[0]) == pytest.approx(float(dtb), rel=1e-12)
    s.close()


@pytest.mark.parametrize("r,rk", [(1, "ssp3"), (2, "imex"), (3, "ssp3"), (3, "imex")])
def test_steps_paper(r, rk):
    say(f"case: 20 steps, paper quadrature, two levels, wet/dry, tracer sources r={r} rk={rk}")
    o, b = coastal_paper(r, rk)
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    for _ in range(20):
        o.step()
        s.step()
    s.sync()
    assert s.diagnostics()["t"] == pytest.approx(o.t, rel=1e-12)
    compare_states(o, s, TOL_STEP, "20 steps")
    s.close()


def vortex_pair(N, r, rk):
    m = Mesh.uniform(2 * N, N, 0.0, 0.0, 1.0 / N, bc=("state", "open", "wall", "wall"))
    o = Oracle(m, Params(r=r, S=(r + 2,), rule="gll", rk=rk, eps=1e-3, h_lim=0.0, adapt_degree=False,
                         quadrature="paper"))
    b = np.zeros(len(o.node_coords()))
    o.set_bathymetry(b)
    return m, o, gpu_from_oracle(o, b)


def exact_fn(v, t):
    def fn(x, y):
        h, u, w = v.fields(x, y, t)
        return h, h * u, h * w, np.zeros_like(x)
    return fn


def l2_errors_state(st, m, r, v, T):
    """L2 errors of zeta and q at time T on a Gauss-Legendre rule of r + 4
    points per direction (the oracle test's measure)."""
    ng = r + 4
    xg, wg = gl_rule(ng)
    X, Y = np.tile(xg, ng), np.repeat(xg, ng)
    B, _, _ = tensor_basis(r, X, Y)
    z, qx, qy = (st[f] @ B.T for f in range(3))
    xs = m.xc[:, None] + X[None] * m.dx[:, None]
    ys = m.yc[:, None] + Y[None] * m.dx[:, None]
    he, ue, ve = v.fields(xs, ys, T)
    w = np.outer(wg, wg).ravel()[None] * m.dx[:, None] ** 2
    return (math.sqrt(np.sum(w * (z - he) ** 2)),
            math.sqrt(np.sum(w * ((qx - he * ue) ** 2 + (qy - he * ve) ** 2))))


@pytest.mark.parametrize("rk,r,cfl,tol", [("rk32", 1, 0.2, 0.03), ("ssp3", 2, 0.1, 0.03), ("rk44", 3, 0.1, 0.005)])
def test_vortex_paper_table7(rk, r, cfl, tol):
    N, T = 20, 1.0 / 6.0
    say(f"case: vortex N={N}, paper quadrature, {rk} r={r}: 10 steps vs the oracle, whole run vs Table 7")
    m, o, s = vortex_pair(N, r, rk)
    v = Vortex()
    K = m.K
    init = l2_project(m, r, lambda x, y: exact_fn(v, 0.0)(x, y)[:3])
    o.set_state(*init)
    s.set_state(*init)
    n = int(math.ceil(T / (cfl / N / (6.9 + math.sqrt(9.81)))))
    dt = T / n
    for k in range(10):
        o.set_boundary_state(exact_fn(v, k * dt))
        s.set_boundary_state(exact_fn(v, k * dt))
        o.step(dt)
        s.step(dt)
    s.sync()
    for f, name in enumerate(("zeta", "qx", "qy")):
        e = rel(cpu(s.get_state()[f], K), o.get_state()[f])
        say(f"  10 steps {name} rel err {e:.3e}")
        assert e < TOL_STEP, (name, e)
    for k in range(10, n):
        s.set_boundary_state(exact_fn(v, k * dt))
        s.step(dt)
    s.sync()
    st = [cpu(x, K) for x in s.get_state()[:3]]
    ez, eq = l2_errors_state(st, m, r, v, T)
    pz, pq = table7()[(rk, r, N)]
    say(f"  {n} steps: L2 zeta {ez:.4e} (Table 7 {pz:.4e}), q {eq:.4e} ({pq:.4e})")
    assert abs(ez / pz - 1.0) < tol and abs(eq / pq - 1.0) < tol, (ez, pz, eq, pq)
    s.close()


def test_paper_argument_checks():
    from paper_2505_18743_amd import Solver
    say("case: paper quadrature argument checks")
    m = Mesh.uniform(4, 3, 0.0, 0.0, 1.0)
    base = dict(r=2, S=(4,), rule="gll", rk="ssp3", quadrature="paper")
    for bad in (dict(S=(5,)), dict(rule="eq"), dict(S=(4, 6))):
        q = dict(base)
        q.update(bad)
        with pytest.raises(RuntimeError, match="paper's quadrature"):
            Solver(mesh_dict(m), q, device="cuda:0")
    s = Solver(mesh_dict(m), base, device="cuda:0")
    n = len(s.node_coords())
    assert n == m.K * (16 + 16)
    s.set_bathymetry(np.full(n, -1.0))
    s.set_manning(np.zeros(m.K))
    z = np.ones((m.K, 9))
    s.set_state(z, 0 * z, 0 * z)
    with pytest.raises(RuntimeError, match="SW_QUAD_PAPER"):
        s.vjp_operator(z, 0 * z, 0 * z, z, z, z)
    s.close()
