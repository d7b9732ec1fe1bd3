"""GPU: given-data boundaries (state and discharge sides) against the oracle:
face-node coordinates, residuals on a hanging mesh with a tracer, steps of the
paper's vortex set-up (exact state at the inflow, open outflow, walls) and of
a channel with a given inflow discharge and an imposed outflow elevation, the
residual VJP with such sides, and the argument checks.
"""
import numpy as np
import pytest
import torch

from exact import Vortex
from oracle import Mesh, Oracle, Params
from oracle.adjoint import residual_vjp
from test_gpu_parity import TOL_RHS, TOL_STEP, cpu, gpu_from_oracle, hanging_case, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def given_fn(x, y):
    return (0.1 * np.sin(y / 300.0), 0.3 + 0.1 * np.cos(x / 200.0), 0.05 + 0.0 * x, 0.7 + 0.1 * np.sin(x / 500.0))


def oracle_nodes(o):
    xs, ys = [], []
    for bg in o.bface_groups:
        if bg["kind"] in ("state", "discharge"):
            xs.append(np.ravel(bg["xy"][0]))
            ys.append(np.ravel(bg["xy"][1]))
    return np.stack([np.concatenate(xs), np.concatenate(ys)], 1)


def sorted_rows(a):
    a = np.round(a, 9)
    return a[np.lexsort((a[:, 1], a[:, 0]))]


@pytest.mark.parametrize("r,S", [(1, (8, 4)), (2, (16, 8))])
def test_boundary_nodes_and_residuals_hanging_tracer(r, S):
    say(f"case: state + discharge sides, hanging mesh, tracer, r={r} S={S}")
    o, b = hanging_case(r, S, bc=("state", "discharge", "wall", "state"))
    o.set_boundary_state(given_fn)
    s = gpu_from_oracle(o, b)
    xy, mem = s.boundary_nodes()
    ref = oracle_nodes(o)
    assert xy.shape == ref.shape and np.all(mem == 0)
    assert np.abs(sorted_rows(xy) - sorted_rows(ref)).max() < 1e-9
    with pytest.raises(RuntimeError, match="boundary"):
        s.apply_operator(*o.get_state(), 0.0)
    s.set_boundary_state(given_fn)
    rng = np.random.default_rng(3)
    st = o.get_state()
    st = [st[0], rng.uniform(-0.5, 0.5, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape), st[3]]
    F, Gx, Gy, R, dtb = o.apply_operator(st, 100.0)
    g = s.apply_operator(st[0], st[1], st[2], st[3], 100.0)
    s.sync()
    K = o.m.K
    for name, gg, rr in (("F", g[0], F), ("Gx", g[1], Gx), ("Gy", g[2], Gy), ("R", g[3], R)):
        e = rel(cpu(gg, K), rr)
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_RHS, (name, e)
    assert float(g[4].cpu()[0]) == pytest.approx(float(dtb), rel=1e-12)
    # 10 steps
    s.set_state(*o.get_state())
    for _ in range(10):
        o.step()
        s.step()
    s.sync()
    for f, name in enumerate(("eta", "qx", "qy", "c")):
        e = rel(cpu(s.get_state()[f], K), o.get_state()[f])
        say(f"  10 steps {name} rel err {e:.3e}")
        assert e < TOL_STEP
    s.close()


def test_vortex_exact_inflow_steps():
    say("case: vortex, exact state at the west inflow, open east, walls, r=2 GLL, 16x8, 40 steps")
    N = 8
    m = Mesh.uniform(2 * N, N, 0.0, 0.0, 1.0 / N, bc=("state", "open", "wall", "wall"))
    p = Params(r=2, S=(5,), rule="gll", rk="ssp3", eps=1e-3, h_lim=0.0, cfl=0.9, cfl_mode=1, adapt_degree=False)
    o = Oracle(m, p)
    b = np.zeros(len(o.node_coords()))
    o.set_bathymetry(b)
    v = Vortex()

    def given(x, y):
        h, u, w = v.fields(x, y, 0.0)
        return h, h * u, h * w, np.zeros_like(x)

    o.set_boundary_state(given)
    d = o.dof_coords()
    h, u, w = v.fields(d[..., 0], d[..., 1], 0.0)
    o.set_state(h, h * u, h * w)
    s = gpu_from_oracle(o, b)
    s.set_boundary_state(given)
    s.set_state(*o.get_state())
    for _ in range(40):
        o.step()
        s.step()
    s.sync()
    for f, name in enumerate(("h", "qx", "qy")):
        e = rel(cpu(s.get_state()[f], o.m.K), o.get_state()[f])
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_STEP
    assert s.diagnostics()["t"] == pytest.approx(o.t, rel=1e-12)
    s.close()


def test_channel_inflow_discharge_steps():
    """Sec. 4.3's channel set-up on a coarse mesh: discharge given at the west
    inflow, zeta = 0 imposed at the east outflow, walls north and south,
    obstacles below the grid scale and Manning friction."""
    say("case: channel, discharge inflow + elevation outflow, r=3, 10x2 cells, S=16, 60 steps")
    L, q0 = 100.0, 0.18
    m = Mesh.uniform(10, 2, 0.0, 0.0, L / 10, bc=("discharge", "elev", "wall", "wall"))
    p = Params(r=3, S=(16,), rule="eq", rk="ssp3", eps=1e-3, h_lim=1e-3, cfl=0.9, cfl_mode=1,
               tide=(0.0, 1.0, 0.0, 0.0))
    o = Oracle(m, p)
    xy = o.node_coords()
    x = xy[:, 0]
    zb0, c0 = 0.2, 1.0
    zb = 4.9 + 0.001 * x - zb0 / 2 * (np.tanh((x - 0.4 * L) / c0) - np.tanh((x - 0.5 * L) / c0)) \
        - zb0 / 4 * (np.tanh((x - 0.55 * L) / c0) - np.tanh((x - 0.6 * L) / c0))
    b = -zb
    o.set_bathymetry(b)
    o.set_manning(np.full(m.K, 0.03))
    o.set_boundary_state(lambda x, y: (np.zeros_like(x), np.full_like(x, q0), np.zeros_like(x), np.zeros_like(x)))
    d = o.dof_coords()
    o.set_state(np.zeros(d.shape[:2]), np.full(d.shape[:2], q0), np.zeros(d.shape[:2]))
    s = gpu_from_oracle(o, b)
    s.set_boundary_state(lambda x, y: (np.zeros_like(x), np.full_like(x, q0), np.zeros_like(x), np.zeros_like(x)))
    s.set_state(*o.get_state())
    m0 = o.total_mass()
    for _ in range(60):
        o.step()
        s.step()
    s.sync()
    got = [cpu(x, o.m.K) for x in s.get_state()[:3]]
    ref = o.get_state()
    # the transverse discharge is a small by-product (the exact discharge mass
    # matrix against the residuals' sample rule), so q is compared as a vector
    qs = max(np.abs(ref[1]).max(), np.abs(ref[2]).max())
    errs = (rel(got[0], ref[0]), np.abs(got[1] - ref[1]).max() / qs, np.abs(got[2] - ref[2]).max() / qs)
    for name, e in zip(("zeta", "qx", "qy"), errs):
        say(f"  {name} rel err {e:.3e}")
        assert e < TOL_STEP
    say(f"  mass {m0:.6f} -> {o.total_mass():.6f} (open boundaries)")
    s.close()


def test_vjp_operator_with_given_sides():
    say("case: vjp_operator, state + discharge sides, hanging mesh")
    o, b = hanging_case(2, (16, 8), tracer=False, bc=("state", "discharge", "wall", "open"))
    o.set_boundary_state(given_fn)
    rng = np.random.default_rng(8)
    K = o.m.K
    o.set_manning(rng.uniform(0.01, 0.04, K))
    o.set_bed_offset(rng.uniform(-0.02, 0.02, K))
    s = gpu_from_oracle(o, b)
    s.set_bed_offset(o.dbed.numpy())
    s.set_boundary_state(given_fn)
    st = o.get_state()
    st = [st[0] + rng.uniform(-0.05, 0.05, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape),
          rng.uniform(-0.5, 0.5, st[0].shape)]
    bars = [rng.standard_normal((K, o.np_)) for _ in range(3)]
    ref = residual_vjp(o, st, 300.0, *bars, o.nman.numpy(), o.dbed.numpy())
    got = s.vjp_operator(st[0], st[1], st[2], bars[0], bars[1], bars[2], 300.0)
    s.sync()
    for name, g_, r_ in zip(("eta_b", "qx_b", "qy_b", "n_bar", "db_bar"), got, ref):
        e = rel(g_.detach().cpu().numpy().reshape(r_.shape), r_)
        say(f"  {name} rel err {e:.3e}")
        assert e < 1e-12, (name, e)
    s.close()


def test_set_boundary_state_errors():
    say("case: boundary data argument checks")
    o, b = hanging_case(1, (8, 4), tracer=False)
    s = gpu_from_oracle(o, b)
    assert len(s.boundary_nodes()[0]) == 0
    with pytest.raises(RuntimeError, match="no state or discharge"):
        s.set_boundary_state(np.zeros((4, 0)))
    s.close()
    o, b = hanging_case(1, (8, 4), tracer=False, bc=("state", "wall", "wall", "wall"))
    s = gpu_from_oracle(o, b)
    n = len(s.boundary_nodes()[0])
    assert n > 0
    with pytest.raises(ValueError):
        s.set_boundary_state(np.zeros((4, n - 1)))
    s.close()
