"""Pins of the oracle's given-data boundaries (state and discharge sides).

* free stream: a uniform flow with every side given that same flow has zero
  residuals (any wrong component, sign or normal in the ghost breaks it);
* lake at rest over a varying bed with the rest state given (Prop. 3.1);
* closed-form face integrals of the Rusanov flux at a discharge inflow into a
  fluid at rest, and at an outflow (tracer taken from inside);
* the travelling vortex (Sec. 4.4) with the exact state given at the inflow,
  an open outflow and walls, as the paper sets it up: design order.
"""
import math

import numpy as np
import pytest

from exact import Vortex
from oracle import Mesh, Oracle, Params, gl_rule, tensor_basis

G = 9.81


def make(mesh, p, depth):
    o = Oracle(mesh, p)
    xy = o.node_coords()
    o.set_bathymetry(-np.asarray(depth(xy[:, 0], xy[:, 1])))
    return o


def test_free_stream_with_given_sides():
    m = Mesh.uniform(4, 3, 0.0, 0.0, 0.5, bc=("state", "open", "discharge", "state"))
    o = make(m, Params(r=2, S=(6,), rule="eq", eps=1e-3, tracer=True), lambda x, y: np.full_like(x, 1.5))
    z0, qx0, qy0, c0 = 0.2, 0.7, -0.3, 0.4
    o.set_boundary_state(lambda x, y: (np.full_like(x, z0), np.full_like(x, qx0), np.full_like(x, qy0),
                                       np.full_like(x, c0)))
    n = (m.K, o.np_)
    st = [np.full(n, z0), np.full(n, qx0), np.full(n, qy0), np.full(n, c0)]
    F, Gx, Gy, R, _ = o.apply_operator(st, 0.0)
    for name, v in (("F", F), ("Gx", Gx), ("Gy", Gy), ("R", R)):
        assert np.abs(v).max() < 1e-13, (name, np.abs(v).max())


def test_lake_at_rest_with_given_state():
    m = Mesh.uniform(3, 3, 0.0, 0.0, 1.0, bc=("state", "state", "discharge", "wall"))
    o = make(m, Params(r=2, S=(8,), rule="eq", eps=1e-3, tracer=True),
             lambda x, y: 2.0 + 0.5 * np.sin(3 * x) * np.cos(2 * y) + 0.3 * (x > 1.4))
    o.set_boundary_state(lambda x, y: (np.full_like(x, 0.1), np.zeros_like(x), np.zeros_like(x),
                                       np.full_like(x, 0.25)))
    n = (m.K, o.np_)
    st = [np.full(n, 0.1), np.zeros(n), np.zeros(n), np.full(n, 0.25)]
    F, Gx, Gy, R, _ = o.apply_operator(st, 0.0)
    for name, v in (("F", F), ("Gx", Gx), ("Gy", Gy), ("R", R)):
        assert np.abs(v).max() < 1e-12, (name, np.abs(v).max())


@pytest.mark.parametrize("side", ["west", "east"])
def test_discharge_face_closed_form(side):
    """Flat wet bed (depth h0), fluid at rest with tracer 0, discharge (qin, 0)
    and tracer 1 given on one side, walls elsewhere.  Only that side's face
    fluxes act; with zeta+ = zeta- the Rusanov mass term reduces to the
    average of the normal discharges, lambda = qin/h0 + sqrt(g h0):
      sum F  = -n_x qin Ly / 2,
      sum Gx = (-n_x qin^2/(2 h0) + lambda qin / 2) Ly  (pressure terms vanish),
      sum R  = (-n_x qin/2 + lambda h0/2) Ly on inflow (n_x = -1), 0 on outflow."""
    h0, qin, Ly = 2.0, 0.8, 1.5
    bc = ("discharge", "wall", "wall", "wall") if side == "west" else ("wall", "discharge", "wall", "wall")
    m = Mesh.uniform(2, 3, 0.0, 0.0, 0.5, bc=bc)
    o = make(m, Params(r=2, S=(5,), rule="eq", eps=1e-3, tracer=True), lambda x, y: np.full_like(x, h0))
    o.set_boundary_state(lambda x, y: (np.full_like(x, 9.0), np.full_like(x, qin), np.zeros_like(x),
                                       np.ones_like(x)))
    n = (m.K, o.np_)
    z = np.zeros(n)
    F, Gx, Gy, R, _ = o.apply_operator([z, z, z, z], 0.0)
    nx = -1.0 if side == "west" else 1.0
    lam = qin / h0 + math.sqrt(G * h0)
    assert F.sum() == pytest.approx(-nx * qin * Ly / 2, rel=1e-13)
    assert Gx.sum() == pytest.approx((-nx * qin ** 2 / (2 * h0) + lam * qin / 2) * Ly, rel=1e-13)
    assert abs(Gy.sum()) < 1e-13
    Rref = (-nx * qin / 2 + lam * h0 / 2) * Ly if nx < 0 else 0.0
    assert R.sum() == pytest.approx(Rref, rel=1e-13, abs=1e-13)


def vortex_state_error(N, r, S, T=0.05, cfl=0.1):
    """The paper's vortex set-up: exact state given at the west inflow, open
    (supercritical) outflow at the east, walls north and south."""
    m = Mesh.uniform(2 * N, N, 0.0, 0.0, 1.0 / N, bc=("state", "open", "wall", "wall"))
    p = Params(r=r, S=(S,), rule="gll", rk="ssp3", eps=1e-3, h_lim=0.0, cfl=cfl, adapt_degree=False)
    o = make(m, p, lambda x, y: np.zeros_like(x))
    v = Vortex()

    def given(x, y):
        h, u, w = v.fields(x, y, 0.0)
        return h, h * u, h * w, np.zeros_like(x)

    o.set_boundary_state(given)
    d = o.dof_coords()
    h, u, w = v.fields(d[..., 0], d[..., 1], 0.0)
    o.set_state(h, h * u, h * w)
    dt0 = cfl * (1.0 / N) / (6.9 + math.sqrt(G))
    nst = int(math.ceil(T / dt0))
    for _ in range(nst):
        o.step(T / nst)
    xg, wg = gl_rule(r + 3)
    X, Y = np.tile(xg, r + 3), np.repeat(xg, r + 3)
    B, _, _ = tensor_basis(r, X, Y)
    z = o.state[0].numpy() @ B.T
    xs = m.xc[:, None] + X[None] * m.dx[:, None]
    ys = m.yc[:, None] + Y[None] * m.dx[:, None]
    he, _, _ = v.fields(xs, ys, T)
    w2 = np.outer(wg, wg).ravel()
    return math.sqrt(np.sum(w2[None] * m.dx[:, None] ** 2 * (z - he) ** 2))


def test_vortex_with_exact_inflow_state_design_order():
    e1 = vortex_state_error(8, 2, 5)
    e2 = vortex_state_error(16, 2, 5)
    assert math.log2(e1 / e2) > 2.8, (e1, e2)
