"""Reference adjoint (vector-Jacobian products) of the all-wet time stepper.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

The paper has no adjoint; this module differentiates the paper's method where
it is differentiable in the ordinary sense.  In the all-wet regime -- every
rule node wet at the start of the step and in every stage, every cell of
degree r (min depth >= h_lim when degree adaptation is on), no tracer -- the
land-sea mask is constant, the depth integral H(zeta) of eq:depth_rhs is
affine in zeta, and the Newton solve of eq:newton reaches the exact solution
of H(zeta) = T in one iteration (the paper notes the one-iteration case).
A step of the explicit Butcher scheme (Sec. 3.1) is then

    H(zeta^(l)) = H(zeta^n) + dt sum_m a_lm F(u^(m))        (eq:algebraic_elevation)
    M q^(l)     = M q^n     + dt sum_m a_lm G(u^(m))        (eq:algebraic_discharge)

with F, G the weak residuals of ``Oracle.residual`` and M the exact discharge
mass matrix, a smooth map of the state and of the per-cell parameters
(Manning n_K, bed offset db_K) away from the kinks of max/min/|.| in the
fluxes.  The solves are written out (H(zeta) = M0 zeta + B with the all-wet
rule mass matrix M0 and B = sum_q W_q psi zb_q) and torch autograd takes the
reverse pass (a library routine used as one step).  Kinks take the branch the
forward took (torch.where semantics): pos(x) has derivative 1 iff x > 0, ties
of max/min go to the first argument, d|x| = sign(x) with sign(0) = 0.

The functions are pinned in tests by: equality of ``allwet_step`` with
``Oracle.step`` on all-wet states; central finite differences of the observed
loss along random directions; and the dot-product identity between the
residual's VJP and its finite-difference directional derivative.
"""
from __future__ import annotations

import numpy as np
import torch

from .swdg import DT, Oracle, tableau, tensor_basis


def regime_ok(o: Oracle, state, dbed, start=True):
    """True when every rule node is wet and, for the start-of-step state with
    degree adaptation on, every cell keeps degree r (min depth >= h_lim,
    eq:criteria_p)."""
    zeta = state[0]
    for lv in o.levels:
        s = zeta[lv.idx] @ lv.Bv.T + o.zb_eff(lv, dbed)
        if bool((s <= 0).any()):
            return False
        if start and o.p.adapt_degree and bool((s.min(1).values < o.p.h_lim).any()):
            return False
    return True


def _rule_mass(o: Oracle, lv):
    """All-wet mass matrix of the sample rule, sum_q W_q psi_i psi_j, per level."""
    return (lv.Bv.T * lv.W) @ lv.Bv


def allwet_step(o: Oracle, state, t, dt, dbed, nman, check=True):
    """One step of the Butcher scheme in the all-wet regime (see module doc).

    ``state`` = [zeta, qx, qy] tensors [K, NP]; ``dbed``, ``nman`` per-cell
    tensors (may require grad).  Returns the new [zeta, qx, qy] and the list
    of stage states."""
    if o.p.tracer:
        raise ValueError("the all-wet adjoint reference has no tracer")
    A, b, c = tableau(o.p.rk)
    s = len(b)
    K = o.m.K
    zeros = torch.zeros(K, o.np_, dtype=DT)
    jac = torch.as_tensor(o.m.dx ** 2, dtype=DT)
    Mq = o.Mq_ref[None] * jac[:, None, None]

    def H_of(zeta):
        """eq:depth_rhs in the all-wet regime: H_i = sum_q W_q psi_i (zeta_q + zb_q)."""
        H = zeros
        for lv in o.levels:
            h = zeta[lv.idx] @ lv.Bv.T + o.zb_eff(lv, dbed)
            H = H.index_add(0, lv.idx, (lv.W * h) @ lv.Bv)
        return H

    def solve_H(T):
        """zeta with H(zeta) = T: M0 zeta = T - B per cell."""
        z = zeros
        for lv in o.levels:
            B = (lv.W * o.zb_eff(lv, dbed)) @ lv.Bv
            M0 = _rule_mass(o, lv)
            rhs = (T[lv.idx] - B).T
            z = z.index_add(0, lv.idx, torch.linalg.solve(M0, rhs).T)
        return z

    zeta, qx, qy = state
    Hn = H_of(zeta)
    Qxn = torch.einsum("kij,kj->ki", Mq, qx)
    Qyn = torch.einsum("kij,kj->ki", Mq, qy)
    stages = []
    res = []
    cur = [zeta, qx, qy]
    for l in range(s + 1):
        if l > 0:
            coef = A[l] if l < s else b
            upto = l if l < s else s
            acc = [zeros, zeros, zeros]
            for m in range(upto):
                if coef[m] != 0.0:
                    acc = [acc[f] + coef[m] * res[m][f] for f in range(3)]
            nz = solve_H(Hn + dt * acc[0])
            nqx = torch.linalg.solve(Mq, (Qxn + dt * acc[1]).unsqueeze(-1)).squeeze(-1)
            nqy = torch.linalg.solve(Mq, (Qyn + dt * acc[2]).unsqueeze(-1)).squeeze(-1)
            cur = [nz, nqx, nqy]
        if l < s:
            if check and not regime_ok(o, [x.detach() for x in cur], dbed.detach(), start=(l == 0)):
                raise ValueError("state left the all-wet regime")
            stages.append(cur)
            F, Gx, Gy, _, _ = o.residual(cur + [zeros], t + c[l] * dt, dbed=dbed, nman=nman)
            res.append((F, Gx, Gy))
    return cur, stages


def point_operator(o: Oracle, xy):
    """Evaluation of a nodal field at points: (cell index, basis values [G, NP])
    so that value_g = sum_j phi[g, j] field[cell[g], j]."""
    m = o.m
    xy = np.asarray(xy, dtype=np.float64)
    x0c = m.x0 + m.ii * m.dx
    y0c = m.y0 + m.jj * m.dx
    cells = np.zeros(len(xy), dtype=np.int64)
    phi = np.zeros((len(xy), o.np_))
    for g, (x, y) in enumerate(xy):
        inside = np.nonzero((x >= x0c) & (x < x0c + m.dx) & (y >= y0c) & (y < y0c + m.dx))[0]
        if len(inside) != 1:
            raise ValueError(f"point {g} is not inside exactly one cell")
        k = int(inside[0])
        cells[g] = k
        v, _, _ = tensor_basis(o.p.r, np.array([(x - x0c[k]) / m.dx[k]]), np.array([(y - y0c[k]) / m.dx[k]]))
        phi[g] = v[0]
    return cells, phi


def observed_run(o: Oracle, state0, t0, dt, nsteps, cells, phi, dbed, nman, check=True):
    """Free-surface values at the points after each of nsteps all-wet steps:
    tensor [nsteps, G]."""
    cells_t = torch.as_tensor(cells, dtype=torch.long)
    phi_t = torch.as_tensor(phi, dtype=DT)
    st = [torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(o.m.K, o.np_) for x in state0[:3]]
    obs = []
    t = t0
    for _ in range(nsteps):
        st, _ = allwet_step(o, st, t, dt, dbed, nman, check=check)
        t = t + dt
        obs.append((st[0][cells_t] * phi_t).sum(1))
    return torch.stack(obs, 0)


def misfit_loss(obs, truth):
    """sum over steps and points of the squared free-surface misfit."""
    return ((obs - truth) ** 2).sum()


def adjoint_gradients(o: Oracle, state0, t0, dt, nsteps, cells, phi, truth, nman, dbed):
    """Loss and its gradients with respect to the per-cell Manning coefficients
    and bed offsets (reverse mode through ``observed_run``)."""
    n = torch.as_tensor(np.asarray(nman, dtype=np.float64)).clone().requires_grad_(True)
    d = torch.as_tensor(np.asarray(dbed, dtype=np.float64)).clone().requires_grad_(True)
    obs = observed_run(o, state0, t0, dt, nsteps, cells, phi, d, n)
    loss = misfit_loss(obs, torch.as_tensor(truth, dtype=DT))
    gn, gd = torch.autograd.grad(loss, (n, d))
    return float(loss.detach()), gn.numpy(), gd.numpy()


def residual_vjp(o: Oracle, state, t, Fb, Gxb, Gyb, nman, dbed):
    """VJP of the weak residuals (F, Gx, Gy) of ``Oracle.residual`` (no tracer):
    returns (zeta_bar, qx_bar, qy_bar, n_bar, db_bar) for the adjoint inputs."""
    K, NP = o.m.K, o.np_
    st = [torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(K, NP).clone().requires_grad_(True)
          for x in state[:3]]
    n = torch.as_tensor(np.asarray(nman, dtype=np.float64)).clone().requires_grad_(True)
    d = torch.as_tensor(np.asarray(dbed, dtype=np.float64)).clone().requires_grad_(True)
    F, Gx, Gy, _, _ = o.residual(st + [torch.zeros(K, NP, dtype=DT)], t, dbed=d, nman=n)
    bars = [torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(K, NP) for x in (Fb, Gxb, Gyb)]
    obj = (F * bars[0]).sum() + (Gx * bars[1]).sum() + (Gy * bars[2]).sum()
    g = torch.autograd.grad(obj, st + [n, d])
    return [x.numpy() for x in g]
