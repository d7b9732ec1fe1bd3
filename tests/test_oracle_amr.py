"""Pins of the oracle's dynamic h-adaptivity (Sec. 3.3 criteria; Sec. 3.4
conservative remap, eq:cons-remap, and the mass source Q^n, eq:mass-loss).

* Indicators against closed forms: a solid-body rotation u = W (-y, x) has
  vorticity 2 W everywhere, also over a sloping free surface (h linear, q =
  h u quadratic, so the chain-rule term of 1/h_des is exercised); inside the
  desingularised layer (h < eps) the vorticity equals a central difference
  of the pointwise u = q / h_des; a linear tracer has a constant gradient.
* Transfer: a child carries its parent's polynomial exactly (checked at
  random points); merging the four children of a refined cell returns the
  cell's own coefficients; a merge keeps the integral of every field and
  leaves a residual orthogonal to Q_r of the parent (the L2 projection).
* Per-cell scalars: refining and merging back returns them exactly; a
  merge keeps their sum over the four children.
* Criteria and 2:1 balance: one flagged cell gives exactly four children;
  flags next to coarse cells force the closure the balance needs and nothing
  more (brute force over all 2:1-balanced refinements of a small mesh); a
  merge that would break the balance is dropped; random flags on random
  quadtrees always give a balanced mesh that contains every flagged split.
* Raster sampling: bilinear functions are reproduced exactly on a raster
  with nx != ny and dx != dy (an i / j or x / y swap fails), raster nodes
  give their values, and points outside take the value at the nearest point
  of the raster (clamping per coordinate).
* Q^n: over a fully wet lake on a rough raster bed, the change of total mass
  across a remesh equals the difference of the bathymetry integrals
  (eq:mass-loss), computed separately from the raster samples.
* The travelling vortex of Sec. 4.4 with AMR (RK32, r = 1, n_max = 2,
  theta_c = 5e-5, theta_r = 1e-4, remesh every 5 steps): its L2 errors equal
  those of the static mesh at the finest level within 0.5 % with fewer than
  half the degrees of freedom, as Table 7 reports.
"""
import math
import itertools

import numpy as np
import pytest
import torch

from exact import G, Vortex
from oracle import Mesh, Oracle, Params, gl_rule, tensor_basis
from oracle.amr import (TRACER_GRAD, VORTICITY, indicator, plan, remesh, sample_raster, transfer,
                        transfer_cellwise, transfer_tables)
from test_oracle_paper_quadrature import l2_errors, l2_project


def flat_oracle(m, r=2, eps=1e-3, **kw):
    o = Oracle(m, Params(r=r, S=(r + 2,) * 4, rule="gll", eps=eps, h_lim=0.0, adapt_degree=False, **kw))
    o.set_bathymetry(np.full(len(o.node_coords()), -1.0))   # depth z_b = 1
    return o


def interp_state(o, fz, fqx, fqy, fc=None):
    d = o.dof_coords()
    x, y = d[..., 0], d[..., 1]
    return [fz(x, y), fqx(x, y), fqy(x, y), fc(x, y) if fc else np.zeros_like(x)]


def test_raster_sampling_is_bilinear_and_clamped():
    rng = np.random.default_rng(7)
    nx, ny, x0, y0, dx, dy = 7, 4, -3.0, 10.0, 2.5, 0.75
    f = lambda x, y: 1.5 - 0.4 * x + 2.0 * y + 0.3 * x * y
    X, Y = np.meshgrid(x0 + dx * np.arange(nx), y0 + dy * np.arange(ny))   # b[j, i]
    grid = dict(x0=x0, y0=y0, dx=dx, dy=dy, b=f(X, Y))
    # interior points: exact for a bilinear function
    xy = np.stack([rng.uniform(x0, x0 + dx * (nx - 1), 200), rng.uniform(y0, y0 + dy * (ny - 1), 200)], axis=1)
    assert np.allclose(sample_raster(grid, xy), f(xy[:, 0], xy[:, 1]), rtol=0.0, atol=1e-12)
    # the raster's own nodes, the last row and column included
    nodes = np.stack([X.ravel(), Y.ravel()], axis=1)
    assert np.allclose(sample_raster(grid, nodes), grid["b"].ravel(), rtol=0.0, atol=1e-13)
    # outside: the value at the nearest raster point, coordinate by coordinate
    out = np.array([[x0 - 5.0, y0 + 1.1], [x0 + dx * (nx - 1) + 3.0, y0 - 2.0], [x0 + 4.2, y0 + dy * ny + 9.0]])
    near = np.stack([np.clip(out[:, 0], x0, x0 + dx * (nx - 1)), np.clip(out[:, 1], y0, y0 + dy * (ny - 1))], axis=1)
    assert np.allclose(sample_raster(grid, out), f(near[:, 0], near[:, 1]), rtol=0.0, atol=1e-12)
    # a non-bilinear raster is matched at the nodes only: a point between
    # nodes is the weighted mean of its four corners
    b2 = rng.uniform(-1, 1, (ny, nx))
    g2 = dict(grid, b=b2)
    p = np.array([[x0 + 2.25 * dx, y0 + 1.5 * dy]])
    want = 0.75 * 0.5 * b2[1, 2] + 0.25 * 0.5 * b2[1, 3] + 0.75 * 0.5 * b2[2, 2] + 0.25 * 0.5 * b2[2, 3]
    assert abs(sample_raster(g2, p)[0] - want) <= 1e-14


@pytest.mark.parametrize("quad", ["subgrid", "paper"])
def test_vorticity_of_solid_body_rotation(quad):
    m = Mesh.uniform(3, 2, 0.0, 0.0, 1.0)
    W = 0.7
    o = flat_oracle(m, r=2, quadrature=quad)
    # free surface zeta = 0.1 x - 0.2 y, depth h = 1 + zeta, q = h W (-y, x)
    h = lambda x, y: 1.0 + 0.1 * x - 0.2 * y
    st = interp_state(o, lambda x, y: 0.1 * x - 0.2 * y, lambda x, y: -W * y * h(x, y),
                      lambda x, y: W * x * h(x, y))
    eta = indicator(o, VORTICITY, st)
    assert np.abs(eta - 2 * W).max() < 1e-12


def test_vorticity_in_the_desingularised_layer():
    m = Mesh.uniform(1, 1, 0.0, 0.0, 1.0)
    eps = 0.5
    o = flat_oracle(m, r=2, eps=eps)
    zeta = lambda x, y: -0.7 + 0.1 * x + 0.05 * y          # h = 0.3 + 0.1 x + 0.05 y < eps
    qx = lambda x, y: 0.2 + 0.3 * y * y - 0.1 * x
    qy = lambda x, y: -0.1 + 0.4 * x * y
    st = interp_state(o, zeta, qx, qy)
    eta = indicator(o, VORTICITY, st)

    def u(x, y):
        hh = zeta(x, y) + 1.0
        ih = math.sqrt(2.0) * hh / math.sqrt(max(hh ** 4, eps ** 4) + hh ** 4)
        return qx(x, y) * ih, qy(x, y) * ih
    xs = o.levels[0].xh
    best = 0.0
    d = 1e-5
    for a in xs:
        for b in xs:
            dvx = (u(a + d, b)[1] - u(a - d, b)[1]) / (2 * d)
            duy = (u(a, b + d)[0] - u(a, b - d)[0]) / (2 * d)
            best = max(best, abs(dvx - duy))
    assert abs(eta[0] - best) < 1e-8 * best


def test_tracer_gradient_indicator():
    m = Mesh.uniform(2, 2, 0.0, 0.0, 2.0)
    o = flat_oracle(m, r=1, tracer=True)
    st = interp_state(o, lambda x, y: 0 * x, lambda x, y: 0 * x, lambda x, y: 0 * x, lambda x, y: 3 * x - 4 * y)
    assert np.abs(indicator(o, TRACER_GRAD, st) - 5.0).max() < 1e-12


@pytest.mark.parametrize("r", [1, 2, 3])
def test_child_carries_the_parent_polynomial(r):
    rng = np.random.default_rng(r)
    child, _ = transfer_tables(r)
    u = rng.normal(size=(r + 1) ** 2)
    X, Y = rng.uniform(size=20), rng.uniform(size=20)
    for s in range(4):
        sx, sy = s & 1, s >> 1
        uc = child[s] @ u
        vc = tensor_basis(r, X, Y)[0] @ uc
        vp = tensor_basis(r, (sx + X) / 2, (sy + Y) / 2)[0] @ u
        assert np.abs(vc - vp).max() < 1e-12


@pytest.mark.parametrize("r", [1, 2, 3])
def test_merge_is_the_l2_projection(r):
    rng = np.random.default_rng(10 + r)
    child, proj = transfer_tables(r)
    u = rng.normal(size=(r + 1) ** 2)
    # restriction followed by the merge is the identity
    assert np.abs(sum(proj[s] @ (child[s] @ u) for s in range(4)) - u).max() < 1e-12
    # four unrelated children: integral kept, residual orthogonal to Q_r(parent)
    kids = [rng.normal(size=(r + 1) ** 2) for _ in range(4)]
    up = sum(proj[s] @ kids[s] for s in range(4))
    ng = r + 3
    xg, wg = gl_rule(ng)
    X, Y = np.tile(xg, ng), np.repeat(xg, ng)
    w = np.outer(wg, wg).ravel() / 4.0
    B = tensor_basis(r, X, Y)[0]
    total_c = 0.0
    res = np.zeros((r + 1) ** 2)
    for s in range(4):
        sx, sy = s & 1, s >> 1
        vc = B @ kids[s]
        Bp = tensor_basis(r, (sx + X) / 2, (sy + Y) / 2)[0]
        total_c += float(w @ vc)
        res += Bp.T @ (w * (vc - Bp @ up))
    xq, wq = gl_rule(ng)
    total_p = float(np.outer(wq, wq).ravel() @ (tensor_basis(r, np.tile(xq, ng), np.repeat(xq, ng))[0] @ up))
    assert abs(total_c - total_p) < 1e-13 * max(1.0, abs(total_c))
    assert np.abs(res).max() < 1e-13


def leaves_of(m):
    return {(int(L), int(i), int(j)) for L, i, j in zip(m.level, m.ii, m.jj)}


def test_one_flag_gives_four_children():
    m = Mesh.uniform(3, 3, 0.0, 0.0, 1.0)
    eta = np.zeros(9)
    eta[4] = 1.0
    nm, rel, nref, ncoa, emax = plan(m, eta, 0.5, 0.0, 3)
    assert nm.K == 12 and nref == 1 and ncoa == 0 and emax == 1.0
    assert leaves_of(nm) == (leaves_of(m) - {(0, 1, 1)}) | {(1, 2 + a, 2 + b) for a in (0, 1) for b in (0, 1)}
    assert [r_[0] for r_ in rel].count("child") == 4
    # ordered by level, then j, then i
    keys = list(zip(nm.level, nm.jj, nm.ii))
    assert keys == sorted(keys)


def test_cell_values_survive_refine_and_merge():
    # per-cell scalars (Manning, bed offset): children inherit, a parent takes
    # the mean of its four children, so refining and merging back returns the
    # original values exactly, and a merge of distinct values keeps their sum
    m = Mesh.uniform(4, 3, 0.0, 0.0, 1.0)
    vals = np.linspace(0.011, 0.04, m.K)
    eta = np.zeros(m.K)
    eta[[1, 6, 10]] = 1.0
    nm, rel, nref, _, _ = plan(m, eta, 0.5, 0.0, 3)
    assert nref == 3
    v1 = transfer_cellwise(vals, rel)
    # merge every refined cell back: children far below theta_c eta_max,
    # n_max = 1 so that nothing refines
    back, rel2, _, ncoa, _ = plan(nm, (nm.level == 0).astype(float), 0.5, 0.1, 1)
    assert ncoa == 3 and back.K == m.K
    assert np.array_equal(transfer_cellwise(v1, rel2), vals)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.01, 0.05, nm.K)
    w2 = transfer_cellwise(w, rel2)
    for n, r_ in enumerate(rel2):
        if r_[0] == "parent":
            assert abs(4.0 * w2[n] - sum(w[k] for k in r_[1])) <= 1e-15


def balanced(leaves, nx0, ny0):
    try:
        Mesh(nx0, ny0, 0.0, 0.0, 1.0, [c[0] for c in leaves], [c[1] for c in leaves], [c[2] for c in leaves])
        return True
    except ValueError:
        return False


def test_closure_is_the_smallest_balanced_refinement():
    # a 2 x 2 coarse grid with one cell split; flag a child in the corner
    # next to the unsplit coarse cells: its split needs the closure
    lv = [0, 0, 0, 1, 1, 1, 1]
    ii = [1, 0, 1, 0, 1, 0, 1]
    jj = [0, 1, 1, 0, 0, 1, 1]
    m = Mesh(2, 2, 0.0, 0.0, 1.0, lv, ii, jj)
    k = [n for n in range(m.K) if (lv[n], ii[n], jj[n]) == (1, 1, 1)][0]
    eta = np.zeros(m.K)
    eta[k] = 1.0
    nm, _, nref, _, _ = plan(m, eta, 0.5, 0.0, 4)
    got = leaves_of(nm)
    assert balanced(sorted(got), 2, 2)
    # brute force: every balanced mesh reachable by splitting cells that
    # contains the flagged split has at least as many leaves
    base = leaves_of(m)
    must = base - {(1, 1, 1)} | {(2, 2 + a, 2 + b) for a in (0, 1) for b in (0, 1)}
    cands = [c for c in must if c[0] == 0]
    best = None
    for pick in itertools.product((0, 1), repeat=len(cands)):
        s = set(must)
        for c, f in zip(cands, pick):
            if f:
                s.discard(c)
                s |= {(1, 2 * c[1] + a, 2 * c[2] + b) for a in (0, 1) for b in (0, 1)}
        if balanced(sorted(s), 2, 2) and (best is None or len(s) < len(best)):
            best = s
    assert got == best and nref == 3


def test_merge_dropped_when_it_breaks_the_balance():
    # level-1 block at the west next to a level-2 block: merging the level-1
    # siblings would face level-2 cells
    leaves = {(1, a, b) for a in (0, 1) for b in (0, 1)}
    leaves |= {(2, 4 + a, b) for a in range(2) for b in range(4)}
    leaves |= {(1, 3, 0), (1, 3, 1)}
    leaves = sorted(leaves)
    m = Mesh(2, 1, 0.0, 0.0, 1.0, [c[0] for c in leaves], [c[1] for c in leaves], [c[2] for c in leaves])
    eta = np.array([0.0 if c[0] == 1 and c[1] < 2 else 1.0 for c in leaves])
    eta[-1] = 1.0
    nm, _, _, ncoa, _ = plan(m, eta, 2.0, 0.5, 3)
    assert ncoa == 0 and leaves_of(nm) == leaves_of(m)
    # everything flagged: the fine block merges, the west block is still
    # held back by the level-2 cells it faces before the merges; a second
    # remesh merges it
    ones = np.ones(len(leaves))
    nm2, _, _, ncoa2, _ = plan(m, ones, 2.0, 1.5, 3)
    assert ncoa2 == 2 and (0, 0, 0) not in leaves_of(nm2) and balanced(sorted(leaves_of(nm2)), 2, 1)
    assert all(c[0] == 1 for c in leaves_of(nm2))
    nm3, _, _, ncoa3, _ = plan(nm2, np.ones(nm2.K), 2.0, 1.5, 3)
    assert ncoa3 == 2 and leaves_of(nm3) == {(0, 0, 0), (0, 1, 0)}


def test_random_flags_keep_the_balance():
    rng = np.random.default_rng(4)
    from workloads import quadtree_desc
    for trial in range(12):
        sel = rng.integers(0, 3, size=2)

        def refine(L, cand):
            return [c for c in cand if (c[1] * 7 + c[2] * 3 + trial) % (3 + sel[0]) == 0]
        d = quadtree_desc(5, 4, 0.0, 0.0, 1.0, refine, 2)
        m = Mesh(d["nx0"], d["ny0"], 0.0, 0.0, 1.0, d["level"], d["i"], d["j"])
        eta = rng.uniform(size=m.K)
        nm, rel, _, _, _ = plan(m, eta, 0.7, 0.3, 4)      # Mesh() raises when unbalanced
        flagged = {(int(m.level[k]), int(m.ii[k]), int(m.jj[k])) for k in range(m.K)
                   if eta[k] > 0.7 * eta.max() and m.level[k] + 1 < 4}
        new = leaves_of(nm)
        assert not (flagged & new)                      # every flagged cell was split
        area = sum(4.0 ** -L for L, _, _ in new)
        assert abs(area - 20.0) < 1e-12


def test_mass_change_is_the_bathymetry_integral_difference():
    rng = np.random.default_rng(2)
    grid = dict(x0=0.0, y0=0.0, dx=0.05, dy=0.05, b=-2.0 + 0.5 * rng.uniform(size=(41, 81)))
    m = Mesh.uniform(8, 4, 0.0, 0.0, 0.5)
    o = Oracle(m, Params(r=2, S=(6, 6), rule="gll", eps=1e-3, h_lim=0.0, adapt_degree=False))
    o.set_bathymetry(sample_raster(grid, o.node_coords()))
    o.set_state(np.full((m.K, 9), 0.25), np.zeros((m.K, 9)), np.zeros((m.K, 9)))
    eta = np.zeros(m.K)
    eta[[3, 9, 10, 20]] = 1.0
    n, rel, st = remesh(o, grid, VORTICITY, 0.5, 0.0, 3, eta=eta)
    assert st["n_refined"] == 4 and n.m.K == m.K + 12

    def bathy_integral(orc):
        tot = 0.0
        for lv in orc.levels:
            tot += float((lv.W * orc.zb_eff(lv)).sum())
        return tot
    dq = bathy_integral(n) - bathy_integral(o)
    assert abs(dq) > 1e-4                                  # the raster is rough: Q^n is not zero
    assert abs(st["q_bathy"] - dq) < 1e-12 * abs(bathy_integral(o))
    assert abs((st["mass_new"] - st["mass_old"]) - dq) < 1e-12 * st["mass_old"]


def vortex_static_and_amr(nmax, r=1, rk="rk32", cfl=0.2, N=20):
    T = 1.0 / 6.0
    v = Vortex()
    grid = dict(x0=-1.0, y0=-1.0, dx=4.0, dy=3.0, b=np.zeros((2, 2)))

    def exact(t):
        return lambda x, y: (lambda h, u, w: (h, h * u, h * w, np.zeros_like(x)))(*v.fields(x, y, t))
    Nf = N * 2 ** (nmax - 1)
    n = int(math.ceil(T / (cfl / Nf / (6.9 + math.sqrt(G)))))
    dt = T / n
    p = Params(r=r, S=(r + 2,) * nmax, rule="gll", rk=rk, eps=1e-3, h_lim=0.0, adapt_degree=False,
               quadrature="paper")
    bc = ("state", "open", "wall", "wall")
    out = {}
    for mode in ("static", "amr"):
        m = Mesh.uniform(2 * (Nf if mode == "static" else N), Nf if mode == "static" else N, 0.0, 0.0,
                         1.0 / (Nf if mode == "static" else N), bc=bc)
        o = Oracle(m, Params(**{**p.__dict__, "S": (r + 2,)}) if mode == "static" else p)
        o.set_bathymetry(np.zeros(len(o.node_coords())))
        o.set_state(*l2_project(m, r, lambda x, y: exact(0.0)(x, y)[:3]))
        if mode == "amr":   # adapt the initial mesh to the initial state, n_max - 1 times
            for _ in range(nmax - 1):
                o, _, _ = remesh(o, grid, VORTICITY, 1e-4, 5e-5, nmax)
                o.set_state(*l2_project(o.m, r, lambda x, y: exact(0.0)(x, y)[:3]))
        for k in range(n):
            if mode == "amr" and k > 0 and k % 5 == 0:
                o, _, st = remesh(o, grid, VORTICITY, 1e-4, 5e-5, nmax)
                assert abs(st["mass_new"] - st["mass_old"]) < 1e-12 * st["mass_old"]   # flat bed: Q^n = 0
            o.set_boundary_state(exact(k * dt))
            o.step(dt)
        out[mode] = l2_errors(o, o.m, r, v, T) + (o.m.K * (r + 1) ** 2 * 3,)
    return out


def test_vortex_amr_matches_the_static_finest_mesh():
    out = vortex_static_and_amr(2)
    (sz, sq, sd), (az, aq, ad) = out["static"], out["amr"]
    assert abs(az / sz - 1.0) < 5e-3 and abs(aq / sq - 1.0) < 5e-3, out
    assert ad < 0.5 * sd, out
