"""Pins of the oracle's linear reactions that couple tracers: the source
h phi_k(c_1, ..., c_M) of eq:shw with phi_k = sum_j B_kj c_j, taken with the
explicit tableau in every stage as eq:imex_shw takes the reactions
(oracle.step_coupled).

* Uniform tracers in a fluid at rest: the step is the linear map of the
  scheme on c' = B c, the stability function R(z) = 1 + z b^T (I - z A)^-1 1
  applied to dt B through B's eigendecomposition, for a lower-triangular B
  (real, distinct eigenvalues; B and its transpose give different results);
  SSP3 converges to expm(B t) c0 at third order.
* B = -kappa I on a moving flow equals each tracer's own first-order decay
  (tracer_decay = kappa, the term inside the residual) to round-off.
* A conversion chain (columns of B summing to zero) on a moving flow in a
  closed basin keeps the total tracer mass sum_k int h c_k to round-off while
  moving mass between the tracers; the same step with B transposed (rows
  summing to zero) does not.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import Mesh, Oracle, Params, step_coupled, tableau

B3 = np.array([[-0.05, 0.0, 0.0],
               [0.03, -0.02, 0.0],
               [0.01, 0.02, -0.01]])


def at_rest(M, rk="ssp3", dx=1000.0, h0=2.0):
    out = []
    for _ in range(M):
        m = Mesh.uniform(2, 2, 0.0, 0.0, dx)
        o = Oracle(m, Params(r=1, S=(4,), rule="eq", rk=rk, eps=1e-3, h_lim=1e-3, tracer=True, adapt_degree=False))
        o.set_bathymetry(np.full(len(o.node_coords()), -h0))
        out.append(o)
    return out


def moving(M, rk="ssp3", **tr):
    """A Gaussian hump of water on a flat 6 m deep basin with walls, r = 2,
    and tracers of different shapes."""
    out = []
    for k in range(M):
        m = Mesh.uniform(4, 3, 0.0, 0.0, 50.0)
        o = Oracle(m, Params(r=2, S=(6,), rule="gll", rk=rk, eps=1e-3, h_lim=1e-3, tracer=True,
                             adapt_degree=False, cfl=0.3, **tr))
        o.set_bathymetry(np.full(len(o.node_coords()), -6.0))
        d = o.dof_coords()
        x, y = d[..., 0], d[..., 1]
        zeta = 0.5 * np.exp(-((x - 80.0) ** 2 + (y - 70.0) ** 2) / 900.0)
        c = 1.0 + 0.5 * np.sin((k + 1) * x / 40.0) * np.cos(y / 30.0)
        z = np.zeros_like(zeta)
        o.set_state(zeta, z, z, c)
        out.append(o)
    return out


def stability(rk, z):
    A, b, _ = tableau(rk)
    A, b = np.array(A, dtype=float), np.array(b, dtype=float)
    s = len(b)
    return 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))


def tracer_mass(o):
    return float(o.conserved()[1].sum())


@pytest.mark.parametrize("rk", ["fe", "ssp3", "rk32", "rk44", "imex"])
def test_uniform_tracers_step_is_the_stability_function_of_dt_B(rk):
    dt, c0 = 2.0, np.array([0.8, 0.3, 0.1])
    os_ = at_rest(3, rk=rk)
    K, NP = os_[0].m.K, os_[0].np_
    z = np.zeros((K, NP))
    for o, c in zip(os_, c0):
        o.set_state(z, z, z, np.full((K, NP), c))
    step_coupled(os_, B3, dt)
    lam, V = np.linalg.eig(B3)
    want = (V @ np.diag([stability(rk, dt * l) for l in lam]) @ np.linalg.inv(V) @ c0).real
    got = np.array([o.get_state()[3] for o in os_])
    for k in range(3):
        assert np.allclose(got[k], want[k], rtol=1e-13, atol=0.0), (k, got[k].ravel()[0], want[k])
    # the transposed matrix is a different map on these values
    wrong = (V @ np.diag([stability(rk, dt * l) for l in lam]) @ np.linalg.inv(V)).real.T @ c0
    assert np.abs(wrong - want).max() > 1e-4


def test_coupled_ssp3_converges_to_the_matrix_exponential():
    T, c0 = 20.0, np.array([1.0, 0.5, 0.2])
    exact = scipy.linalg.expm(B3 * T) @ c0
    errs = []
    for dt in (4.0, 2.0, 1.0):
        os_ = at_rest(3)
        K, NP = os_[0].m.K, os_[0].np_
        z = np.zeros((K, NP))
        for o, c in zip(os_, c0):
            o.set_state(z, z, z, np.full((K, NP), c))
        for _ in range(int(round(T / dt))):
            step_coupled(os_, B3, dt)
        errs.append(max(abs(o.get_state()[3][0, 0] - e) for o, e in zip(os_, exact)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 2.8, (errs, rates)


@pytest.mark.parametrize("rk", ["ssp3", "imex"])
def test_diagonal_reactions_are_the_decay(rk):
    kappa, dt = 4e-3, 0.5
    coupled = moving(2, rk=rk)
    own = moving(2, rk=rk, tracer_decay=kappa)
    for _ in range(5):
        step_coupled(coupled, -kappa * np.eye(2), dt)
        for o in own:
            o.step(dt)
    for a, b in zip(coupled, own):
        ca, cb = a.get_state()[3], b.get_state()[3]
        assert np.abs(ca - cb).max() <= 1e-13 * np.abs(cb).max()
        # and the flow is the same as without any tracer source
        for f in range(3):
            assert np.array_equal(a.get_state()[f], b.get_state()[f])


def test_conversion_chain_keeps_the_total_tracer_mass():
    a, b, dt = 0.05, 0.04, 0.5
    chain = np.array([[-a, 0.0, 0.0], [a, -b, 0.0], [0.0, b, 0.0]])   # c1 -> c2 -> c3
    assert np.allclose(chain.sum(axis=0), 0.0)

    def run(B):
        os_ = moving(3)
        m0 = [tracer_mass(o) for o in os_]
        for _ in range(8):
            step_coupled(os_, B, dt)
        return m0, [tracer_mass(o) for o in os_]

    m0, m1 = run(chain)
    assert abs(sum(m1) - sum(m0)) <= 1e-13 * sum(m0)
    assert m1[0] < m0[0] * (1 - 0.1) and m1[2] > m0[2] * (1 + 0.05)
    # a planted mistake: the transpose converts along rows and changes the total
    t0, t1 = run(chain.T)
    assert abs(sum(t1) - sum(t0)) > 1e-4 * sum(t0)
