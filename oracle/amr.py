"""Dynamic h-adaptivity of the oracle: the refinement indicator and criteria
of Sec. 3.3 ("Degree and h-adaptivity"), the conservative remap of the state
onto the new quadtree (eq:cons-remap) and the spurious mass source Q^n of
bathymetry re-sampling (eq:mass-loss), Sec. 3.4.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the product path
never imports it, and it shares no code with the HIP library.

Readings (where the paper is silent they are the oracle's choices, listed in
the design notes too):
  * Indicator nodes: the nodes of the volume integrals, the Gaussian rule of
    Table 1 with the paper's quadrature and the S x S sample rule otherwise;
    both carry bathymetry samples, which the depth needs.
  * Vorticity indicator (Sec. 4.4): eta_K = max over the nodes of
    |d_x u_y - d_y u_x| with u = q / h_des (eq:velocity), differentiated by
    the chain rule; the depth gradient is taken as grad zeta at wet nodes,
    since the bed is known by its samples only (exact on a flat bed), and a
    dry node gives zero.  Tracer indicator (Sec. 5): eta_K = max |grad c|.
  * Criteria: refine K if eta_K > theta_r eta_max, n_K < n_max and the cell
    size exceeds H_min; coarsen if eta_K < theta_c eta_max and n_K > 1, with
    n_K = level + 1.  Four siblings merge only when all four are leaves,
    all flagged for coarsening and none is refined.  The mesh stays 2:1
    balanced across faces (the hanging faces the method supports):
    refinement wins, a leaf two or more levels coarser than a face neighbour
    is refined until none is left, and a merge that would leave a face
    neighbour two levels finer is dropped.
  * Transfer: the L2 projection onto Q_r of the new cells, which keeps the
    integral of every field over every old cell group (eq:cons-remap).  A
    child takes its parent's polynomial (exact); a parent takes the
    projection of its four children with the exact mass matrix.  zeta, q and
    c are remapped; a child inherits the Manning coefficient and bed offset,
    a parent takes the mean of its children's.  New cells start at degree r
    (the next step decides degrees, Sec. 3.3).
  * The remesh acts on the state after the degree decision and remap that
    start the next step (what the library holds between steps).
  * Bathymetry of the new cells: sampled from a raster by bilinear
    interpolation ("extracted from a bathymetry database"), clamped to the
    raster's edge outside it.
  * New cells are ordered by level, then row j, then column i.
  * Q^n (eq:mass-loss): sum over new cells of int z_b l minus the same over
    the old cells, on the sample rule, with l the land-sea mask of the state
    on each mesh; the total masses before and after are reported beside it.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .swdg import DT, BC_PERIODIC, Mesh, Oracle, _Vol, _inv_des, _pos, basis_nodes, gl_rule, tensor_basis

VORTICITY, TRACER_GRAD = "vorticity", "tracer_grad"


def sample_raster(grid, xy):
    """Bilinear interpolation of a raster b[j, i] given at (x0 + i dx, y0 + j dy),
    i < nx, j < ny (nx, ny >= 2), clamped to the raster outside it."""
    b = np.asarray(grid["b"], dtype=np.float64)
    ny, nx = b.shape
    fx = np.clip((xy[:, 0] - grid["x0"]) / grid["dx"], 0.0, nx - 1.0)
    fy = np.clip((xy[:, 1] - grid["y0"]) / grid["dy"], 0.0, ny - 1.0)
    i0 = np.minimum(np.floor(fx).astype(np.int64), nx - 2)
    j0 = np.minimum(np.floor(fy).astype(np.int64), ny - 2)
    tx, ty = fx - i0, fy - j0
    return ((1.0 - tx) * (1.0 - ty) * b[j0, i0] + tx * (1.0 - ty) * b[j0, i0 + 1]
            + (1.0 - tx) * ty * b[j0 + 1, i0] + tx * ty * b[j0 + 1, i0 + 1])


def _dinv_des(h, eps):
    """d(1/h_des)/dh of eq:velocity: -1/h^2 for h >= eps, sqrt(2) (eps^4 - h^4)
    (eps^4 + h^4)^(-3/2) for 0 < h < eps, 0 on dry nodes."""
    e4 = eps ** 4
    h4 = h ** 4
    thin = math.sqrt(2.0) * (e4 - h4) / (e4 + h4) ** 1.5
    hs = torch.where(h > 0, h, torch.ones_like(h))
    return torch.where(h >= eps, -1.0 / hs ** 2, torch.where(h > 0, thin, torch.zeros_like(h)))


def indicator(o: Oracle, kind: str, state=None):
    """eta_K of every cell (see the module notes); state defaults to the one the
    next step starts from."""
    st = o.adapted_state() if state is None else state
    st = [torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(o.m.K, o.np_) for x in st]
    eta = torch.zeros(o.m.K, dtype=DT)
    for lv in o.levels:
        idx = lv.idx
        if len(idx) == 0:
            continue
        vr = lv if lv.vol is None else _Vol(lv.vol)
        zb = o.zb_eff(lv) if lv.vol is None else o.zb_vol_eff(lv)
        Bv, Bx, By = vr.Bv, vr.Bx / lv.dx, vr.By / lv.dx
        if kind == VORTICITY:
            Z, QX, QY = st[0][idx], st[1][idx], st[2][idx]
            s = Z @ Bv.T + zb
            wet = s > 0
            h = _pos(s)
            qx, qy = QX @ Bv.T, QY @ Bv.T
            ih, dih = _inv_des(h, o.p.eps), _dinv_des(h, o.p.eps)
            hx = torch.where(wet, Z @ Bx.T, torch.zeros_like(h))
            hy = torch.where(wet, Z @ By.T, torch.zeros_like(h))
            curl = ih * (QY @ Bx.T - QX @ By.T) + dih * (qy * hx - qx * hy)
            val = curl.abs()
        elif kind == TRACER_GRAD:
            C = st[3][idx]
            val = torch.sqrt((C @ Bx.T) ** 2 + (C @ By.T) ** 2)
        else:
            raise ValueError(f"unknown indicator {kind!r}")
        eta[idx] = val.max(1).values
    return eta.numpy()


# ---------------------------------------------------------------------------
# The new quadtree
# ---------------------------------------------------------------------------

def _neighbour(m: Mesh, L, i, j, di, dj):
    """Face-neighbour position at level L (periodic sides wrap), None outside."""
    nxL, nyL = m.nx0 << L, m.ny0 << L
    ni, nj = i + di, j + dj
    if not 0 <= ni < nxL:
        if m.bc[0] != BC_PERIODIC:
            return None
        ni %= nxL
    if not 0 <= nj < nyL:
        if m.bc[2] != BC_PERIODIC:
            return None
        nj %= nyL
    return ni, nj


def plan(m: Mesh, eta, theta_r, theta_c, n_max, h_min=0.0):
    """Leaves of the adapted quadtree and, per new leaf, where its state comes
    from: ("copy", k), ("child", k, sx, sy) or ("parent", [k00, k10, k01, k11]).
    Returns (new Mesh, relations, n_refined, n_coarsened, eta_max)."""
    K = m.K
    eta = np.asarray(eta, dtype=np.float64)
    eta_max = float(eta.max()) if K else 0.0
    lev, ii, jj = m.level, m.ii, m.jj
    refine = (eta > theta_r * eta_max) & (lev + 1 < n_max) & (m.dx > h_min)
    coarsen = (eta < theta_c * eta_max) & (lev > 0) & ~refine
    old = {(int(lev[k]), int(ii[k]), int(jj[k])): k for k in range(K)}
    leaves = set(old)
    for k in np.nonzero(refine)[0]:
        key = (int(lev[k]), int(ii[k]), int(jj[k]))
        leaves.discard(key)
        L, i, j = key
        leaves |= {(L + 1, 2 * i + a, 2 * j + b) for a in (0, 1) for b in (0, 1)}
    # 2:1 closure across faces: refine every leaf two or more levels coarser
    # than a face neighbour
    changed = True
    while changed:
        changed = False
        for (L, i, j) in sorted(leaves, reverse=True):
            if (L, i, j) not in leaves:
                continue
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                nb = _neighbour(m, L, i, j, di, dj)
                if nb is None:
                    continue
                for A in range(L - 2, -1, -1):
                    key = (A, nb[0] >> (L - A), nb[1] >> (L - A))
                    if key in leaves:
                        leaves.discard(key)
                        leaves |= {(A + 1, 2 * key[1] + a, 2 * key[2] + b) for a in (0, 1) for b in (0, 1)}
                        changed = True
                        break
    refined = {k for k in old if k not in leaves}
    # merges of four flagged sibling leaves that keep the 2:1 balance
    parents = set()
    for k in np.nonzero(coarsen)[0]:
        L, i, j = int(lev[k]), int(ii[k]), int(jj[k])
        parents.add((L - 1, i >> 1, j >> 1))
    merged = []
    for P in sorted(parents):
        L, pi, pj = P
        kids = [(L + 1, 2 * pi + a, 2 * pj + b) for b in (0, 1) for a in (0, 1)]
        if not all(kd in old and kd in leaves and coarsen[old[kd]] for kd in kids):
            continue
        ok = True
        for side, (di, dj) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
            nb = _neighbour(m, L, pi, pj, di, dj)
            if nb is None:
                continue
            # cells of level L + 2 inside the neighbour square along P's side
            for t in range(4):
                if side == 0:
                    c = (L + 2, 4 * nb[0] + 3, 4 * nb[1] + t)
                elif side == 1:
                    c = (L + 2, 4 * nb[0], 4 * nb[1] + t)
                elif side == 2:
                    c = (L + 2, 4 * nb[0] + t, 4 * nb[1] + 3)
                else:
                    c = (L + 2, 4 * nb[0] + t, 4 * nb[1])
                if c in leaves:
                    ok = False
            if not ok:
                break
        if ok:
            merged.append(P)
    for P in merged:
        L, pi, pj = P
        for a in (0, 1):
            for b in (0, 1):
                leaves.discard((L + 1, 2 * pi + a, 2 * pj + b))
        leaves.add(P)
    new = sorted(leaves, key=lambda c: (c[0], c[2], c[1]))
    rel = []
    for (L, i, j) in new:
        if (L, i, j) in old:
            rel.append(("copy", old[(L, i, j)]))
        elif L > 0 and (L - 1, i >> 1, j >> 1) in old:
            rel.append(("child", old[(L - 1, i >> 1, j >> 1)], i & 1, j & 1))
        else:
            kids = [(L + 1, 2 * i + a, 2 * j + b) for b in (0, 1) for a in (0, 1)]
            if not all(kd in old for kd in kids):
                raise RuntimeError("a new leaf is neither an old leaf, a child nor a parent of old leaves")
            rel.append(("parent", [old[kd] for kd in kids]))
    nm = Mesh(m.nx0, m.ny0, m.x0, m.y0, m.dx0, [c[0] for c in new], [c[1] for c in new], [c[2] for c in new],
              m.bc)
    return nm, rel, len(refined), len(merged), eta_max


# ---------------------------------------------------------------------------
# Conservative transfer (eq:cons-remap)
# ---------------------------------------------------------------------------

def transfer_tables(r):
    """child[s] [n_p, n_p]: nodal values on child s (s = 2 sy + sx) of the
    parent basis, child_u = parent_u @ child[s].T; proj[s] [n_p, n_p]: the
    exact-mass L2 projection's part from child s, parent_u = sum_s child_u_s @ proj[s].T."""
    n1 = r + 1
    xi = basis_nodes(r)
    Xs, Ys = np.tile(xi, n1), np.repeat(xi, n1)
    xg, wg = gl_rule(r + 1)               # exact for the degree-2r products
    Xg, Yg = np.tile(xg, n1), np.repeat(xg, n1)
    wgg = np.outer(wg, wg).ravel()
    Bg = tensor_basis(r, Xg, Yg)[0]
    Mq = Bg.T @ (wgg[:, None] * Bg)       # exact mass matrix of the unit square
    child, proj = [], []
    for s in range(4):
        sx, sy = s & 1, s >> 1
        child.append(tensor_basis(r, (sx + Xs) / 2.0, (sy + Ys) / 2.0)[0])
        Bp = tensor_basis(r, (sx + Xg) / 2.0, (sy + Yg) / 2.0)[0]   # parent basis at the child's nodes
        rhs = Bp.T @ ((0.25 * wgg)[:, None] * Bg)                    # int_child psi_i^P psi_k^child
        proj.append(np.linalg.solve(Mq, rhs))
    return child, proj


def transfer(fields, rel, r):
    """Per-cell arrays [K_old, n_p] -> [K_new, n_p] along the relations."""
    child, proj = transfer_tables(r)
    out = np.zeros((len(rel), fields.shape[1]))
    for n, rr in enumerate(rel):
        if rr[0] == "copy":
            out[n] = fields[rr[1]]
        elif rr[0] == "child":
            out[n] = child[2 * rr[3] + rr[2]] @ fields[rr[1]]
        else:
            out[n] = sum(proj[s] @ fields[k] for s, k in enumerate(rr[1]))
    return out


def transfer_cellwise(values, rel):
    """Per-cell scalars: a child inherits, a parent takes the mean."""
    out = np.zeros(len(rel))
    for n, rr in enumerate(rel):
        out[n] = values[rr[1]] if rr[0] in ("copy", "child") else float(np.mean([values[k] for k in rr[1]]))
    return out


def _mass_terms(o: Oracle, state):
    """Total mass sum int h and sum int z_b l over the sample rule."""
    mass = bathy = 0.0
    for lv in o.levels:
        if len(lv.idx) == 0:
            continue
        s = torch.as_tensor(state[0][lv.idx.numpy()]) @ lv.Bv.T + o.zb_eff(lv)
        wet = s > 0
        mass += float((lv.W * _pos(s)).sum())
        bathy += float((lv.W * torch.where(wet, o.zb_eff(lv), torch.zeros_like(s))).sum())
    return mass, bathy


def remesh(o: Oracle, grid, kind, theta_r, theta_c, n_max, h_min=0.0, eta=None):
    """One remesh: a new Oracle on the adapted mesh with the transferred state,
    Manning coefficients and bed offsets, the bathymetry sampled from the
    raster and the time carried over (boundary data must be given again), and
    the statistics of the step."""
    st = o.adapted_state()
    if eta is None:
        eta = indicator(o, kind, st)
    nm, rel, nref, ncoa, eta_max = plan(o.m, eta, theta_r, theta_c, n_max, h_min)
    n = Oracle(nm, o.p)
    n.set_bathymetry(sample_raster(grid, n.node_coords()))
    n.set_manning(transfer_cellwise(o.nman.numpy(), rel))
    n.set_bed_offset(transfer_cellwise(o.dbed.numpy(), rel))
    new_state = [transfer(np.asarray(x), rel, o.p.r) for x in st]
    n.set_state(*new_state)
    n.t = o.t
    m_old, b_old = _mass_terms(o, st)
    m_new, b_new = _mass_terms(n, new_state)
    stats = dict(n_cells_old=o.m.K, n_cells_new=nm.K, n_refined=nref, n_coarsened=ncoa, eta_max=eta_max,
                 mass_old=m_old, mass_new=m_new, q_bathy=b_new - b_old)
    return n, rel, stats
