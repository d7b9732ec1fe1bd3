"""Pins of the oracle's all-wet adjoint reference (CPU).

* ``allwet_step`` is the paper's step (``Oracle.step``) in the all-wet regime;
* the reverse-mode gradient of the observed misfit matches central finite
  differences of the same loss along random directions;
* the residual VJP satisfies <w, J v> = <J^T w, v> with J v from central
  differences.
"""
import numpy as np
import pytest
import torch

from helpers import build_oracle
from oracle.adjoint import (adjoint_gradients, allwet_step, misfit_loss, observed_run, point_operator,
                            regime_ok, residual_vjp)
from workloads import workload


def small_adjoint_case(n=8, seed=3):
    wl = workload("adjoint_128", n=n)
    o, _ = build_oracle(wl)
    rng = np.random.default_rng(seed)
    _, _, _, _, dtb = o.residual(o.state, 0.0)
    dt = 0.9 * o.p.cfl * float(dtb)
    return wl, o, rng, dt


def test_allwet_step_is_the_paper_step():
    wl, o, rng, dt = small_adjoint_case(10)
    K = o.m.K
    o.set_manning(rng.uniform(0.015, 0.04, K))
    o.set_bed_offset(rng.uniform(-0.05, 0.05, K))
    st = [x.clone() for x in o.state[:3]]
    t = 0.0
    for _ in range(3):
        st, _ = allwet_step(o, st, t, dt, o.dbed, o.nman)
        d = o.step(dt)
        t += dt
        assert d["newton_it"] == 1 and d["n_r0"] == 0
    # the two differ only in rounding: Oracle.step forms the stage increment as
    # M^-1 (T - H(zeta^n)) from depth integrals of ~20 m water, which costs
    # about 1e-16 * |H| / |dt F| ~ 1e-12 relative on the increments
    ref = o.get_state()
    for f in range(3):
        e = np.abs(st[f].numpy() - ref[f]).max() / np.abs(ref[f]).max()
        assert e < 1e-11, (f, e)


def test_regime_check_rejects_dry_states():
    wl, o, rng, dt = small_adjoint_case(6)
    st = [x.clone() for x in o.state[:3]]
    assert regime_ok(o, st, o.dbed)
    st[0] = st[0] - 30.0          # everything dry
    assert not regime_ok(o, st, o.dbed)
    with pytest.raises(ValueError):
        allwet_step(o, st, 0.0, dt, o.dbed, o.nman)


def _loss(o, st0, dt, nsteps, cells, phi, truth, n, d):
    obs = observed_run(o, st0, 0.0, dt, nsteps, cells, phi, torch.as_tensor(d), torch.as_tensor(n))
    return float(misfit_loss(obs, torch.as_tensor(truth)))


def test_misfit_gradient_matches_central_differences():
    """Reverse-mode gradient vs central differences of the same loss (20 steps
    from a flowing state).  The bed offsets alternate in sign between
    neighbours so that no face sits on the min(zb-, zb+) kink within the
    difference step; the loss is the squared free surface at 8 points (a
    misfit against zero) so that it is O(1) and the differences are not lost
    in rounding."""
    wl, o, rng, dt = small_adjoint_case(8)
    K = o.m.K
    nsteps = 20
    L = o.m.nx0 * o.m.dx0
    dxy = o.dof_coords()
    st0 = [o.state[0].clone(), torch.as_tensor(np.sin(2 * np.pi * dxy[..., 1] / L)),
           torch.as_tensor(0.7 * np.cos(2 * np.pi * dxy[..., 0] / L))]
    gauges = rng.uniform(0.1 * L, 0.9 * L, size=(8, 2))
    cells, phi = point_operator(o, gauges)
    truth = np.zeros((nsteps, len(gauges)))
    n0 = np.full(K, 0.0275)
    par = (o.m.ii + o.m.jj) % 2
    d0 = np.where(par == 1, 1e-3, -1e-3) + rng.uniform(-1e-4, 1e-4, K)
    loss, gn, gd = adjoint_gradients(o, st0, 0.0, dt, nsteps, cells, phi, truth, n0, d0)
    assert loss > 0 and np.abs(gn).max() > 0 and np.abs(gd).max() > 0
    h = 1e-5
    for trial in range(3):
        vn = rng.standard_normal(K) * (trial != 1)
        vd = rng.standard_normal(K) * (trial != 0)
        lp = _loss(o, st0, dt, nsteps, cells, phi, truth, n0 + h * vn, d0 + h * vd)
        lm = _loss(o, st0, dt, nsteps, cells, phi, truth, n0 - h * vn, d0 - h * vd)
        fd = (lp - lm) / (2 * h)
        ad = float(gn @ vn + gd @ vd)
        assert abs(fd - ad) <= 2e-4 * abs(ad), (trial, fd, ad)


def test_residual_vjp_dot_product_wet_dry():
    wl = workload("coastal_steps_16")
    o, _ = build_oracle(wl)
    K, NP = o.m.K, o.np_
    rng = np.random.default_rng(11)
    st = o.get_state()
    st = [st[0] + rng.uniform(-0.05, 0.05, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape),
          rng.uniform(-0.5, 0.5, st[0].shape)]
    nman = rng.uniform(0.01, 0.04, K)
    dbed = rng.uniform(-1e-2, 1e-2, K)
    bars = [rng.standard_normal((K, NP)) for _ in range(3)]
    g = residual_vjp(o, st, 0.0, *bars, nman, dbed)

    def R(st_, n_, d_):
        out = o.residual([torch.as_tensor(x) for x in st_] + [torch.zeros(K, NP, dtype=torch.float64)], 0.0,
                         dbed=torch.as_tensor(d_), nman=torch.as_tensor(n_))
        return sum(float((out[f] * torch.as_tensor(bars[f])).sum()) for f in range(3))

    h = 1e-7
    for trial in range(4):
        vs = [rng.standard_normal((K, NP)) * (trial in (0, 3)) for _ in range(3)]
        vn = rng.standard_normal(K) * (trial in (1, 3))
        vd = rng.standard_normal(K) * (trial in (2, 3))
        fp = R([st[f] + h * vs[f] for f in range(3)], nman + h * vn, dbed + h * vd)
        fm = R([st[f] - h * vs[f] for f in range(3)], nman - h * vn, dbed - h * vd)
        fd = (fp - fm) / (2 * h)
        ad = sum(float((g[f] * vs[f]).sum()) for f in range(3)) + float(g[3] @ vn) + float(g[4] @ vd)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (trial, fd, ad)
