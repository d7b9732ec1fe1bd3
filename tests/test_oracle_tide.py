"""Pins of the oracle's elevation boundary (the tide of the coastal set-ups;
boundary ghost of Sec. 3.2 with zeta imposed, q extrapolated and the inflow
tracer value taken where q.n < 0).

* residual of a lake at rest under the imposed elevation at a given time:
  the face integrals are closed forms (Rusanov mass term lambda/2 jump,
  non-conservative pressure g avg(h*) jump, eq:mass_rhs, eq:discharge_rhs);
* the stage times c_l dt of a Butcher step (Sec. 3.1): with a tide of period
  2 dt from a phase of zero, the SSP3 stages see zeta_b = 0, 0 and A, so one
  step moves exactly dt b_3 times the stage-3 face integrals into the domain;
* the tracer ghost: the inflow value on inflow, the interior value on
  outflow (closed-form tracer flux, eq:r_concentration).
"""
import math

import numpy as np
import pytest

from oracle import Mesh, Oracle, Params

G = 9.81


def basin(nx, ny, dx, h0, tide, rk="ssp3", tracer=False, r=1, S=4):
    m = Mesh.uniform(nx, ny, 0.0, 0.0, dx, bc=("elev", "wall", "wall", "wall"))
    o = Oracle(m, Params(r=r, S=(S,), rule="eq", rk=rk, eps=1e-3, h_lim=1e-3, tide=tide, tracer=tracer,
                         adapt_degree=False))
    o.set_bathymetry(-np.full(len(o.node_coords()), h0))
    return o, m


@pytest.mark.parametrize("t", [0.0, 1234.5, 30000.0])
def test_elevation_ghost_lake_at_rest(t):
    A, T, ph = 0.5, 44712.0, 0.3
    h0, dx, ny = 3.0, 100.0, 3
    o, m = basin(2, ny, dx, h0, (A, T, ph, 0.0))
    zb = A * math.sin(2.0 * math.pi * t / T + ph)
    z = np.zeros((m.K, o.np_))
    F, Gx, Gy, R, _ = o.apply_operator([z, z, z, z], t)
    # ghost depth h0 + zb, interior h0: lambda = sqrt(g max(h0, h0 + zb))
    lam = math.sqrt(G * max(h0, h0 + zb))
    l = dx
    assert F.sum() == pytest.approx(ny * 0.5 * lam * zb * l, rel=1e-12, abs=1e-12)
    # west normal (-1, 0): Gx gets + pres n_x with pres = g/2 avg(h*) (0 - zb)
    assert Gx.sum() == pytest.approx(ny * 0.5 * G * (h0 + 0.5 * zb) * zb * l, rel=1e-12, abs=1e-12)
    assert np.abs(Gy).max() < 1e-12
    # only the west cells see the boundary; the flux is spread over their dofs
    west = m.ii == 0
    assert np.abs(F[~west]).max() < 1e-12 and np.abs(F[west]).max() > 1e-3


def test_elevation_ghost_at_stage_times():
    dt, A, h0, dx, ny = 2.0, 0.25, 2.0, 50.0, 2
    o, m = basin(3, ny, dx, h0, (A, 2.0 * dt, 0.0, 0.0))
    z = np.zeros((m.K, o.np_))
    o.set_state(z, z, z)
    m0 = o.total_mass()
    o.step(dt)
    # SSP3: c = (0, 1, 1/2), b3 = 2/3; zeta_b(0) = 0, zeta_b(dt) = A sin(pi) ~ 1e-16 A,
    # zeta_b(dt/2) = A; the stage-3 state is the rest state to O(1e-16)
    lam = math.sqrt(G * (h0 + A))
    dmass = dt * (2.0 / 3.0) * ny * 0.5 * lam * A * dx
    assert o.total_mass() - m0 == pytest.approx(dmass, rel=1e-10)
    qx = o.get_state()[1]
    Jq = o.Mq_ref.numpy().sum(0) * dx * dx          # int psi_j over a cell
    mom = float((qx @ Jq).sum())
    assert mom == pytest.approx(dt * (2.0 / 3.0) * ny * 0.5 * G * (h0 + 0.5 * A) * A * dx, rel=1e-10)
    assert o.t == pytest.approx(dt)


@pytest.mark.parametrize("direction", [1.0, -1.0])
def test_elevation_ghost_tracer_inflow_choice(direction):
    """Uniform state with zeta = the imposed elevation, q = (s q0, 0), tracer
    c0 inside and c_in at the tide boundary (west, n = (-1, 0)).  s = +1 is an
    inflow there (q.n < 0): the ghost takes c_in; s = -1 an outflow: the
    ghost keeps c0.  Sum of R over all cells = minus the west face integral
    of the Rusanov tracer flux (the east wall mirrors q: zero tracer flux;
    interior faces cancel)."""
    A, T, ph, cin = 0.4, 1000.0, math.pi / 2, 0.9   # zeta_b(0) = A exactly
    h0, dx, ny, q0, c0 = 2.0, 10.0, 2, 0.3, 0.2
    o, m = basin(2, ny, dx, h0, (A, T, ph, cin), tracer=True)
    n = (m.K, o.np_)
    st = [np.full(n, A), np.full(n, direction * q0), np.zeros(n), np.full(n, c0)]
    F, Gx, Gy, R, _ = o.apply_operator(st, 0.0)
    h = h0 + A
    lam = q0 / h + math.sqrt(G * h)
    cg = cin if direction > 0 else c0
    qn = -direction * q0                                  # q.n at the west face
    flux = 0.5 * (qn * c0 + qn * cg) + 0.5 * lam * h * (c0 - cg)
    assert R.sum() == pytest.approx(-ny * dx * flux, rel=1e-12)
