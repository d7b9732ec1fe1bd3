"""Pins of the oracle's IMEX friction matrix and of its constant-mode
fallbacks (Sec. 3.1 eq:imex_shw, Sec. 3.2 eq:algebraic_discharge,
eq:mass_matrix_discharge, eq:discharge_rhs_implicit; Sec. 3.3 the singular
land-sea-mask Jacobian).

* The friction-modified discharge matrix takes gamma at the plain depth h of
  the previous stage, the implicit residual L at the desingularised depth:
  for a uniform thin layer (h < eps) on a periodic bed the cell integral of
  the stage-2 discharge is J q0 (1 - chi dt gamma(h_des)) / (1 + chi dt
  gamma(h)), a closed form that a matrix built with h_des misses by 12x in
  gamma.
* A dry node adds nothing to that matrix (gamma q -> 0 at h = 0).
* The IMEX discharge solve of a cell whose matrix is beyond double precision
  (one roundoff-thin node with discharge) takes the degree-0 update
  sum Q / (J + ct int gamma); a well-conditioned cell solves A q = Q.
* Newton on a cell with one wet node: the masked Jacobian is singular
  (rank one), so the constant-mode update shifts zeta by (Hbar - Tbar)/Awet
  and the new cell mass equals the target exactly.
* Tracer on the same cell: the h-weighted matrix is singular, the
  constant-mode update c = c_keep + (sum CT - int h c_keep)/Hbar makes the
  cell's tracer mass int h c equal sum CT.
"""
import math

import numpy as np
import pytest
import torch

from oracle import Mesh, Oracle, Params

G = 9.81


def periodic_flat(h, eps, n, q0, r=1, S=4, rule="eq"):
    m = Mesh.uniform(2, 2, 0.0, 0.0, 100.0, bc=("periodic",) * 4)
    o = Oracle(m, Params(r=r, S=(S,), rule=rule, rk="imex", eps=eps, h_lim=1e-6, adapt_degree=False))
    o.set_bathymetry(-np.full(len(o.node_coords()), h))      # depth h, zeta = 0
    o.set_manning(np.full(m.K, n))
    sh = (m.K, o.np_)
    o.set_state(np.zeros(sh), np.full(sh, q0), np.zeros(sh))
    return o


@pytest.mark.parametrize("rule", ["eq", "gll"])
def test_imex_matrix_takes_plain_depth(rule):
    h, eps, n, q0, dt = 0.05, 0.1, 0.05, 0.01, 1.0
    o = periodic_flat(h, eps, n, q0, rule=rule)
    o.step(dt)
    chi = 1.0 - math.sqrt(2.0) / 2.0
    hdes = math.sqrt(max(h ** 4, eps ** 4) + h ** 4) / (math.sqrt(2.0) * h)   # eq:velocity
    gam_h = G * n * n * q0 / h ** (7.0 / 3.0)
    gam_d = G * n * n * q0 / hdes ** (7.0 / 3.0)
    assert gam_h / gam_d > 10.0
    J = 100.0 ** 2
    q2 = o.last_stages[1][1]                                  # stage-2 qx, nodal
    mean = (q2 @ (o.mean_w * J)).numpy()                      # cell integrals
    want = J * q0 * (1.0 - chi * dt * gam_d) / (1.0 + chi * dt * gam_h)
    assert np.allclose(mean, want, rtol=1e-13, atol=0.0), (mean, want)


def test_imex_friction_terms_vanish_on_dry_nodes():
    m = Mesh.uniform(2, 1, 0.0, 0.0, 10.0, bc=("wall",) * 4)
    o = Oracle(m, Params(r=2, S=(6,), rule="eq", rk="imex", eps=0.1, adapt_degree=False))
    ns = 36                                                   # sample nodes per cell, cell by cell
    o.set_bathymetry(np.concatenate([np.full(ns, 1.0), np.full(ns, -1.0)]))   # cell 0 land, cell 1 depth 1
    o.set_manning(np.full(m.K, 0.03))
    sh = (m.K, o.np_)
    st = [torch.zeros(sh, dtype=torch.float64), torch.full(sh, 0.5, dtype=torch.float64),
          torch.full(sh, -0.2, dtype=torch.float64), torch.zeros(sh, dtype=torch.float64)]
    Lx, Ly, Gam = o._friction(st)
    assert float(Gam[0].abs().max()) == 0.0 and float(Lx[0].abs().max()) == 0.0
    assert float(Ly[0].abs().max()) == 0.0
    # the wet cell: depth 1 >= eps, gamma at h and h_des agree; int gamma = sum Gam
    gam = G * 0.03 ** 2 * math.hypot(0.5, -0.2) / 1.0 ** (7.0 / 3.0)
    assert float(Gam[1].sum()) == pytest.approx(gam * 100.0, rel=1e-13)
    assert float(Lx[1].sum()) == pytest.approx(-gam * 0.5 * 100.0, rel=1e-13)


def test_imex_discharge_solve_and_constant_mode_fallback():
    r, S = 1, 3
    m = Mesh.uniform(2, 1, 0.0, 0.0, 2.0, bc=("wall",) * 4)
    o = Oracle(m, Params(r=r, S=(S,), rule="eq", rk="imex"))
    lv = o.levels[0]
    J = 4.0
    Mq = o.Mq_ref[None] * J
    Mq = Mq.expand(2, -1, -1).clone()
    # cell 0: moderate friction spread over the nodes; cell 1: one node (the
    # centre) with a friction weight 1e30 times the mass
    gam = torch.zeros(2, S * S, dtype=torch.float64)
    gam[0] = torch.linspace(0.1, 0.9, S * S, dtype=torch.float64)
    gam[1, 4] = 1e30
    Gam = torch.einsum("kq,qi,qj->kij", lv.W * gam, lv.Bv, lv.Bv)
    Q = torch.tensor([[1.0, -2.0, 0.5, 3.0], [0.7, 0.2, -0.4, 1.1]], dtype=torch.float64)
    ct = 0.3
    full = torch.ones(2, dtype=torch.bool)
    qx, qy, fb = o._discharge_solve(Mq, torch.full((2,), J, dtype=torch.float64), Gam, ct, Q, -Q, full)
    assert fb.tolist() == [False, True]
    A0 = Mq[0] + ct * Gam[0]
    assert torch.allclose(A0 @ qx[0], Q[0], rtol=0, atol=1e-13 * float(Q[0].abs().max()))
    assert torch.equal(qy[0], -qx[0])
    want = float(Q[1].sum()) / (J + ct * float(Gam[1].sum()))
    assert torch.allclose(qx[1], torch.full((4,), want, dtype=torch.float64), rtol=1e-14, atol=0)
    # a degree-0 cell takes the same formula
    qx0, _, fb0 = o._discharge_solve(Mq, torch.full((2,), J, dtype=torch.float64), Gam, ct, Q, Q,
                                    torch.zeros(2, dtype=torch.bool))
    assert not fb0.any()
    want0 = float(Q[0].sum()) / (J + ct * float(Gam[0].sum()))
    assert torch.allclose(qx0[0], torch.full((4,), want0, dtype=torch.float64), rtol=1e-14, atol=0)


def one_wet_node_cell(tracer=False):
    """One cell, r = 1, the 3 x 3 closed equispaced rule: dry land (bed +10 m)
    except the corner node (0, 0), depth 1 m under zeta = 0.  The basis is
    nodal at the corners, so the masked Jacobian and the tracer matrix are
    W_00 e_0 e_0^T: rank one."""
    m = Mesh.uniform(1, 1, 0.0, 0.0, 4.0, bc=("wall",) * 4)
    o = Oracle(m, Params(r=1, S=(3,), rule="eq", tracer=tracer, adapt_degree=False))
    xy = o.node_coords()
    corner = (xy[:, 0] == 0.0) & (xy[:, 1] == 0.0)
    o.set_bathymetry(np.where(corner, -1.0, 10.0))
    return o


def test_newton_constant_mode_fallback():
    o = one_wet_node_cell()
    lv = o.levels[0]
    W00 = float(lv.W[0])
    assert W00 == pytest.approx(16.0 / 16.0)                 # dx^2 w_0 w_0 = 16 (1/4)^2
    z0 = torch.zeros(1, 4, dtype=torch.float64)
    T = torch.tensor([[0.3, 0.1, 0.05, 0.05]], dtype=torch.float64)   # Tbar = 0.5
    z, its, h, H, Hbar, fb = o._newton(lv, torch.arange(1), T, z0, torch.ones(1, dtype=torch.bool))
    assert bool(fb[0]) and int(its[0]) == 1
    # constant mode: zeta <- zeta - (Hbar - Tbar)/Awet at every node; h_00 = Tbar / W00
    shift = (W00 * 1.0 - 0.5) / W00
    assert torch.allclose(z, torch.full((1, 4), -shift, dtype=torch.float64), rtol=0, atol=1e-15)
    assert float(Hbar[0]) == pytest.approx(0.5, abs=1e-15)


def test_tracer_constant_mode_fallback():
    o = one_wet_node_cell(tracer=True)
    lv = o.levels[0]
    W00 = float(lv.W[0])
    h = torch.zeros(1, 9, dtype=torch.float64)
    h[0, 0] = 0.8
    ck = torch.tensor([[0.2, 0.4, 0.6, 0.8]], dtype=torch.float64)
    CT = torch.tensor([[0.1, 0.3, 0.05, 0.15]], dtype=torch.float64)   # sum 0.6
    c = o._tracer_solve(lv, h, CT, ck, torch.ones(1, dtype=torch.bool))
    Hbar = W00 * 0.8
    want = ck + (0.6 - Hbar * 0.2) / Hbar                    # int h c_keep = Hbar c_keep(x_00)
    assert torch.allclose(c, want, rtol=0, atol=1e-15)
    assert float(Hbar * c[0, 0]) == pytest.approx(0.6, rel=1e-15)   # tracer mass = sum CT
