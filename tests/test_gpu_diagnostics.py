"""GPU: the step's diagnostic outputs and failure modes against the oracle
(positivity violations, Newton iteration counts, constant-mode fallbacks,
non-finite state), each driven on purpose from the host:

* a perched 1 cm layer stepped at 30 times the positivity bound (Props. 3.2,
  3.3): the (cell, stage) pairs with a negative target mass and the smallest
  target equal the oracle's;
* the Newton iteration cap (eq:newton) at a wet/dry front with
  newton_max = 1: the reported maximum and the state equal the oracle's;
* degree adaptation off at a wet/dry front, explicit and IMEX: partially wet
  cells of degree r meet singular land-sea-mask Jacobians (Sec. 3.3), whose
  constant-mode updates are counted step by step like the oracle's;
* a NaN put into the state through sw_set_state: the next step's
  diagnostics report SW_ENONFINITE (a value check, no invalid index).
"""
import numpy as np
import pytest

from helpers import build_oracle
from test_gpu_parity import (TOL_STEP, beach_crop, compare_states, cpu, gpu_from_oracle, rel, solver_for)
from test_oracle_properties import perched_cell

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("rk", ["fe", "ssp3"])
def test_positivity_violation_count(rk):
    say(f"case: perched cell at 30x the positivity bound, {rk}")
    o = perched_cell(rk, 30.0)
    b = -o.levels[0].zb.numpy().ravel()
    s = gpu_from_oracle(o, b)
    s.set_state(*o.get_state())
    d = o.step()
    s.step()
    s.sync()
    dg = s.diagnostics()
    say(f"  oracle n_viol {d['n_viol']} min target {d['min_target']:.6e}; "
        f"gpu {dg['n_pos_viol']} {dg['min_target_mass']:.6e}")
    assert d["n_viol"] > 0
    assert dg["n_pos_viol"] == d["n_viol"]
    assert dg["min_target_mass"] == pytest.approx(d["min_target"], rel=1e-12)
    assert dg["dt"] == pytest.approx(d["dt"], rel=1e-12)
    # the perched cell's target is negative: its Newton solve has no root and
    # leaves it dry, where any zeta <= -max z_b is the same state; the
    # comparison takes H_i and q there (compare_states)
    compare_states(o, s, TOL_STEP, "1 step")
    s.close()


def test_newton_iteration_cap():
    say("case: shore crop 24x12 with a surge, newton_max = 1, 30 steps")
    wl = beach_crop(200, 60, surge=(16200.0, 0.6))
    o, b = build_oracle(wl, newton_max=1)
    s = solver_for(wl, o, b, newton_max=1)
    s.set_state(*o.get_state())
    for k in range(30):
        d = o.step()
        s.step()
        s.sync()
        dg = s.diagnostics()
        assert dg["max_newton_it"] == d["newton_it"] == 1, (k, dg["max_newton_it"], d["newton_it"])
    compare_states(o, s, TOL_STEP, "30 steps")
    s.close()


@pytest.mark.parametrize("rk", ["ssp3", "imex"])
def test_constant_mode_fallbacks_without_degree_adaptation(rk):
    say(f"case: shore crop 24x12 with a surge, adapt_degree = 0, {rk}, 40 steps")
    wl = beach_crop(200, 60, surge=(16200.0, 0.6))
    o, b = build_oracle(wl, adapt_degree=False, rk=rk)
    s = solver_for(wl, o, b, adapt_degree=0, rk=rk)
    s.set_state(*o.get_state())
    tot = 0
    for k in range(40):
        d = o.step()
        s.step()
        s.sync()
        dg = s.diagnostics()
        assert dg["n_fallback"] == d["n_fallback"], (k, dg["n_fallback"], d["n_fallback"])
        assert dg["max_newton_it"] == d["newton_it"], (k, dg["max_newton_it"], d["newton_it"])
        assert dg["n_r0_cells"] == 0
        tot += d["n_fallback"]
    say(f"  constant-mode updates over the run: {tot}")
    assert tot > 0
    compare_states(o, s, TOL_STEP, "40 steps")
    assert dg["total_mass"] == pytest.approx(o.total_mass(), rel=1e-12)
    s.close()


def test_nonfinite_state_is_reported():
    say("case: NaN in qx of one cell through sw_set_state, coastal_steps_16, one step")
    from workloads import workload
    wl = workload("coastal_steps_16")
    o, b = build_oracle(wl)
    s = solver_for(wl, o, b)
    st = o.get_state()
    qx = st[1].copy()
    qx[37, 2] = np.nan
    s.set_state(st[0], qx, st[2])
    s.step(1.0)
    s.sync()
    with pytest.raises(RuntimeError, match="status -4"):
        s.diagnostics()
    # a finite state clears the flag at the next step
    s.set_state(*st[:3])
    s.step(1.0)
    s.sync()
    assert s.diagnostics()["nonfinite"] == 0
    s.close()
