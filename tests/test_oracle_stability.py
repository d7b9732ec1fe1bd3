"""Linear stability of the finest level of the tidal quadtree workload:
degree r = 3 on the 8-point closed equispaced (trapezoid) rule.  The
positivity bound of Prop. 3.2 (dt <= w_1 J / (lambda l), w_1 = 1/14 for this
rule) is not a linear stability bound: a 1 mm hump on a flat 20 m bed grows
without limit at 0.9 x the bound (and at 0.6), while at the workload's
0.4 x the bound it stays a small wave.  The Gauss-Lobatto rule with the same
nodes count runs stably at the same time step, so the loss comes from the
trapezoid rule's under-integration of the degree-3 terms.
"""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params
from workloads import workload


def hump_run(rule, cfl_factor, nsteps, n=12):
    m = Mesh.uniform(n, n, 0.0, 0.0, 50.0)
    o = Oracle(m, Params(r=3, S=(8,), rule=rule, rk="ssp3", eps=0.1, h_lim=0.1, cfl=cfl_factor, cfl_mode=1))
    o.set_bathymetry(np.full(len(o.node_coords()), -20.0))
    o.set_manning(np.full(m.K, 0.025))
    dof = o.dof_coords()
    L = n * 50.0
    eta = 1e-3 * np.exp(-((dof[..., 0] - L / 2) ** 2 + (dof[..., 1] - L / 2) ** 2) / (2.0 * 150.0 ** 2))
    o.init_lake_at_rest(eta)
    qmax = 0.0
    for _ in range(nsteps):
        o.step()
        qmax = max(qmax, float(np.abs(o.get_state()[1]).max()))
        if not np.isfinite(qmax) or qmax > 1.0:
            break
    return qmax


def test_workload_time_step_factor():
    assert workload("tidal_quadtree_r3")["params"]["cfl"] == 0.4


def test_r3_trapezoid8_stable_at_workload_step():
    assert hump_run("eq", 0.4, 150) < 1e-2


def test_r3_trapezoid8_unstable_at_0p9_bound():
    assert hump_run("eq", 0.9, 150) > 1.0


def test_r3_gll8_stable_at_the_same_step():
    # GLL_8 end weight 1/56: factor 3.6 gives the time step of the trapezoid at 0.9
    assert hump_run("gll", 3.6, 150) < 1e-2
