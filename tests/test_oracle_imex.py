"""Pins of the oracle's IMEX step (RK32 explicit companion, TR-BDF2 implicit
companion for the friction, linearised at the previous stage; Sec. 3.1,
eq:imex_shw, eq:algebraic_discharge, eq:mass_matrix_discharge, Appendix A):

* the tableaux satisfy the order and coupling conditions of Appendix A;
* without friction the IMEX step is the RK32 step, bit for bit;
* a uniform flow on a flat periodic bed decays under Manning friction as the
  closed form q(t) = q0 / (1 + kappa q0 t), kappa = g n^2 / h^(7/3), with
  second-order convergence in dt;
* with stiff friction (kappa q0 dt = 12) the IMEX run stays bounded and tends
  to the closed form where the explicit RK32 step diverges;
* mass is conserved to roundoff through a wet/dry dam break with friction.
"""
import math

import numpy as np
import pytest

from helpers import build_oracle
from oracle import Mesh, Oracle, Params, tableau
from oracle.swdg import implicit_tableau
from workloads import workload

G = 9.81


def test_imex_tableaux_order_and_coupling():
    A, b, c = tableau("imex")
    At, bt = implicit_tableau("imex")
    s = len(b)
    chi = 1.0 - math.sqrt(2.0) / 2.0
    assert c[1] == pytest.approx(2.0 * chi, abs=1e-15)
    for l in range(s):
        assert sum(A[l]) == pytest.approx(c[l], abs=1e-15)       # c = row sums, explicit
        assert sum(At[l]) == pytest.approx(c[l], abs=1e-15)      # c~ = c
        assert all(At[l][m] == 0.0 for m in range(l + 1, s))     # DIRK
        assert all(A[l][m] == 0.0 for m in range(l, s))          # explicit
    assert bt == b                                               # preserves linear invariants
    for w in (b, bt):
        assert sum(w) == pytest.approx(1.0, abs=1e-15)
        assert sum(wl * cl for wl, cl in zip(w, c)) == pytest.approx(0.5, abs=1e-15)
    assert At[1][1] == pytest.approx(chi, abs=1e-16) and At[2][2] == pytest.approx(chi, abs=1e-16)


@pytest.mark.parametrize("case", ["coastal", "hanging_tracer"])
def test_imex_without_friction_is_rk32(case):
    if case == "coastal":
        wl = workload("coastal_steps_16")
        o1, _ = build_oracle(wl, rk="rk32")
        o2, _ = build_oracle(wl, rk="imex")
    else:
        from test_gpu_parity import hanging_case
        o1, _ = hanging_case(2, (16, 8))
        o2, _ = hanging_case(2, (16, 8))
        o1.p.rk, o2.p.rk = "rk32", "imex"
        o1.set_manning(np.zeros(o1.m.K))
        o2.set_manning(np.zeros(o2.m.K))
    for _ in range(4):
        o1.step()
        o2.step()
    for x, y in zip(o1.get_state(), o2.get_state()):
        assert np.array_equal(x, y)


def uniform_friction(rk, dt, T, n, h0=1.0, q0=1.0):
    m = Mesh.uniform(2, 2, 0.0, 0.0, 1000.0, bc=("periodic",) * 4)
    o = Oracle(m, Params(r=1, S=(4,), rule="eq", rk=rk, eps=1e-3, h_lim=1e-3, adapt_degree=False))
    o.set_bathymetry(-np.full(len(o.node_coords()), h0))
    o.set_manning(np.full(4, n))
    sh = (4, o.np_)
    o.set_state(np.zeros(sh), np.full(sh, q0), np.zeros(sh))
    out = [q0]
    for _ in range(int(round(T / dt))):
        o.step(dt)
        out.append(float(o.get_state()[1].mean()))
    return np.array(out)


def test_imex_friction_decay_second_order():
    n, T = 0.05, 20.0
    kappa = G * n * n
    exact = 1.0 / (1.0 + kappa * T)
    errs = [abs(uniform_friction("imex", dt, T, n)[-1] - exact) for dt in (1.0, 0.5, 0.25)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, (errs, rates)
    assert errs[-1] < 5e-7


def test_imex_stiff_friction_stays_bounded():
    """kappa q0 dt = 12: the stages take the friction implicitly (linearised at
    the previous stage), the final combination explicitly with b~ = b, so the
    first step overshoots below zero; the run stays bounded by q0 and tends to
    the closed form, where the explicit RK32 step diverges."""
    n, dt, T = 0.5, 5.0, 40.0
    kappa = G * n * n
    assert kappa * dt > 12.0
    q = uniform_friction("imex", dt, T, n)
    assert np.all(np.isfinite(q)) and np.abs(q).max() <= 1.0
    assert np.all(np.abs(q[2:]) < np.abs(q[1:-1]))
    exact = 1.0 / (1.0 + kappa * T)
    assert abs(q[-1] - exact) < 0.3 * exact
    with np.errstate(all="ignore"):
        qe = uniform_friction("rk32", dt, T, n)
    assert not np.all(np.isfinite(qe)) or np.abs(qe).max() > 1e3


def test_imex_mass_conservation_wet_dry():
    wl = workload("beach_dambreak_256", window=(200, 60, 12, 8))
    o, _ = build_oracle(wl, rk="imex")
    m0 = o.total_mass()
    for _ in range(15):
        o.step()
    assert o.total_mass() == pytest.approx(m0, rel=1e-13)


def test_channel_ode_reference_pins():
    """The steady-flow ODE solution of the strong-friction channel: RK4 at two
    resolutions agrees to 1e-9; zeta = 0 at the outflow; the surface rises
    upstream (friction slope); the flow stays subcritical."""
    from channel import G, Q0, depth, steady_profile
    x1, z1 = steady_profile(4000)
    x2, z2 = steady_profile(20000)
    assert abs(z2[-1]) < 1e-14
    assert np.abs(np.interp(x1, x2, z2) - z1).max() < 1e-9
    assert np.all(np.diff(z2) < 0.0)
    h = z2 + depth(x2)
    assert (Q0 ** 2 / (G * h ** 3)).max() < 0.05


def test_imex_channel_runs_beyond_the_explicit_limit():
    """Sec. 4.3, strong friction on the coarsest mesh (N = 10, r = 1): from
    rest, RK32 diverges at dt = 0.02 s, while IMEX runs stably at 2.5 times
    that step (the factor the paper reports) and stays near the steady
    profile; RK32 at dt = 0.01 s is still stable over the same start."""
    from channel import channel_oracle, steady_profile
    def run(rk, dt, n):
        o, _ = channel_oracle(10, 1, rk)
        with np.errstate(all="ignore"):
            for _ in range(n):
                o.step(dt)
                z = o.get_state()[0]
                if not np.all(np.isfinite(z)) or np.abs(z).max() > 1e3:
                    return None
        return o.get_state()[0]
    assert run("rk32", 0.02, 50) is None
    assert run("rk32", 0.01, 150) is not None
    z = run("imex", 0.05, 400)
    assert z is not None
    xe, ze = steady_profile(4000)
    assert z.max() < 1.05 * ze.max() and z.min() > -0.5
