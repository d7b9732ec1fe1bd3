"""Pins of the tracer's numerical diffusion (eq:numdiff, Sec. 3.2) and of a
first-order decay source (the reaction term h phi(c), phi(c) = -kappa c, of
eq:shw, taken with the explicit tableau as eq:imex_shw takes the
reactions):

* decay of a uniform tracer in a fluid at rest: one step of each explicit
  scheme multiplies c by the scheme's stability function
  R(z) = 1 + z b^T (I - z A)^-1 1 at z = -kappa dt (the Butcher tableau's
  linear map, evaluated here by a dense solve), and SSP3 converges to
  exp(-kappa t) at third order;
* the diffusion term of a linear c = c0 + g x in a cell at rest on a flat bed
  is the closed form -nu h g int d_x psi_i = -nu h g (+-dx/2) with
  nu = C |K| S / r^2;
* the term never moves tracer mass between or out of cells (its entries sum
  to zero in every cell) and never adds tracer variance (sum_i c_i D_i <= 0).
"""
import math

import numpy as np
import pytest
import torch

from oracle import Mesh, Oracle, Params, tableau


def at_rest(r=1, S=4, n=2, dx=10.0, h0=2.0, rk="ssp3", **tr):
    m = Mesh.uniform(n, n, 0.0, 0.0, dx)
    o = Oracle(m, Params(r=r, S=(S,), rule="eq", rk=rk, eps=1e-3, h_lim=1e-3, tracer=True, adapt_degree=False, **tr))
    o.set_bathymetry(np.full(len(o.node_coords()), -h0))
    return o, m


def stability(rk, z):
    A, b, _ = tableau(rk)
    A, b = np.array(A, dtype=float), np.array(b, dtype=float)
    s = len(b)
    return 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))


@pytest.mark.parametrize("rk", ["fe", "ssp3", "rk32", "rk44", "imex"])
def test_decay_step_is_the_stability_function(rk):
    kappa, dt, c0 = 0.05, 2.0, 0.8
    o, m = at_rest(rk=rk, dx=1000.0, tracer_decay=kappa)     # gravity-wave CFL 0.02
    sh = (m.K, o.np_)
    o.set_state(np.zeros(sh), np.zeros(sh), np.zeros(sh), np.full(sh, c0))
    o.step(dt)
    c = o.get_state()[3]
    assert np.allclose(c, c0 * stability(rk, -kappa * dt), rtol=1e-13, atol=0.0)


def test_decay_converges_at_third_order():
    kappa, T, c0 = 0.1, 20.0, 1.0
    errs = []
    for dt in (4.0, 2.0, 1.0):
        o, m = at_rest(dx=1000.0, tracer_decay=kappa)
        sh = (m.K, o.np_)
        o.set_state(np.zeros(sh), np.zeros(sh), np.zeros(sh), np.full(sh, c0))
        for _ in range(int(round(T / dt))):
            o.step(dt)
        errs.append(abs(o.get_state()[3][0, 0] - c0 * math.exp(-kappa * T)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 2.8, (errs, rates)


def test_diffusion_of_a_linear_tracer_closed_form():
    C, Sr, h0, dx, g = 0.33, 0.02, 2.0, 10.0, 0.3
    o, m = at_rest(n=1, dx=dx, h0=h0, tracer_diff=C, tracer_strain=Sr)
    dof = o.dof_coords()[0]
    c = 0.5 + g * dof[:, 0]
    z = np.zeros((1, o.np_))
    F, Gx, Gy, R, _ = o.apply_operator([z, z, z, c[None, :]], 0.0)
    nu = C * dx * dx * Sr / 1 ** 2
    sign = np.where(np.isclose(dof[:, 0], dx), 1.0, -1.0)     # +int d_x psi on the east nodes
    assert np.allclose(R[0], -nu * h0 * g * sign * dx / 2.0, rtol=1e-13, atol=1e-15)
    assert np.abs(F).max() == 0.0


@pytest.mark.parametrize("r", [1, 2, 3])
def test_diffusion_keeps_cell_mass_and_dissipates(r):
    rng = np.random.default_rng(r)
    base, _ = at_rest(r=r, S=r + 3, n=3)
    diff, m = at_rest(r=r, S=r + 3, n=3, tracer_diff=0.3, tracer_strain=0.05)
    xy = base.node_coords()
    b = -2.0 - 0.5 * np.sin(xy[:, 0] / 7.0) * np.cos(xy[:, 1] / 4.0)
    base.set_bathymetry(b)
    diff.set_bathymetry(b)
    sh = (m.K, base.np_)
    st = [rng.uniform(-0.2, 0.2, sh), rng.uniform(-0.3, 0.3, sh), rng.uniform(-0.3, 0.3, sh), rng.uniform(0, 1, sh)]
    D = diff.apply_operator(st, 0.0)[3] - base.apply_operator(st, 0.0)[3]
    scale = np.abs(D).max()
    assert scale > 1e-6
    assert np.abs(D.sum(1)).max() < 1e-12 * scale * base.np_
    assert (st[3] * D).sum(1).max() <= 1e-12 * scale
