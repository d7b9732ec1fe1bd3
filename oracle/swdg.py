"""Plain FP64 CPU oracle of the sub-grid-bathymetry DG shallow-water method.

Arpaia, Orlando, Ferrarin, Bonaventura, "High-order adaptive discontinuous
finite elements for the shallow water equations with sub-grid irregular
bathymetry", arXiv:2505.18743.

TEST INFRASTRUCTURE ONLY: this module is the reference the HIP library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does.  It shares no code, table or constant generator with the HIP library.

How it is written
-----------------
Every integral is a direct sum over quadrature nodes of the pointwise
integrand times the basis (or basis-gradient) values at the node, with no
sum factorisation: the basis values at all nodes of a rule form a matrix and a
matmul performs the sum over nodes (a library primitive used as one step).
Per-cell dense solves use torch.linalg (Cholesky).  Everything is float64.
Vectorisation over cells and faces only applies the same per-cell / per-face
definition to many cells at once.

Notation follows the paper: ``zeta`` is the free-surface elevation, ``zb`` the
bathymetry DEPTH (positive downwards), water depth ``h = max(zeta + zb, 0)``
(Sec. 2, eq:zeta2depth-2).  Bed elevation ``b`` as used by callers is ``-zb``.

Readings of the paper that this oracle takes where the text is silent,
ambiguous or garbled (each one is also listed in the design notes):
  * Sub-grid rule: every element integral (volume terms, the continuity mass
    matrix, H, the tracer matrix) uses one closed S x S tensor rule per cell
    whose nodes are the bathymetry samples; face integrals use the rule's
    boundary row, so the face nodes coincide with the mass-rule boundary
    nodes required by the positivity argument (Sec. 3.4, Prop. 3.2).
    The paper's own rules (Table 1) are the special case S = r+2 GLL for the
    mass terms.  The discharge mass matrix is the exact one (Gauss-Legendre
    (r+1)^2, Table 1 / Sec. 3.3).
  * Boundary faces use a ghost state and the interior flux formulas
    (walls mirror the normal discharge; an elevation boundary imposes
    zeta, extrapolates q and takes the inflow tracer value on inflow; a
    state boundary imposes a given (zeta, q, c) at every face node, as for an
    exact solution at a supercritical inflow; a discharge boundary imposes a
    given q, extrapolates zeta and takes the given c where q.n < 0, as for
    the subcritical inflow of a channel).  Given boundary data are held
    constant over a step.
  * Rusanov speed uses the unreconstructed depths (eq:lxf_parameter).
  * Friction is explicit, added to the discharge residual, with the
    desingularised depth (eq:discharge_rhs_implicit with an explicit RK).
    With the IMEX pair the residual L keeps the desingularised depth and the
    friction-modified discharge matrix (eq:mass_matrix_discharge) takes the
    plain depth h of the previous stage, as printed; a dry node (h = 0) adds
    nothing to that matrix.  A cell whose friction-modified matrix fails the
    Cholesky pivot test below takes the degree-0 (constant-mode) discharge
    update for that stage.
  * Newton stop (eq:newton and the text after eq:mass_matrix): the paper stops
    on an l1 increment below 1e-16.  Because H is piecewise linear in zeta,
    an iterate whose land-sea mask equals the previous iterate's mask is the
    exact root (the next increment is exactly zero in exact arithmetic); the
    oracle stops on that event, on the paper's 1e-16 test, or after
    ``newton_max`` iterations.
  * A masked mass matrix whose Cholesky pivot falls below 1e-14*trace is
    replaced by a constant-mode (mass-only) update for that iteration.
  * Dry-cell initial guess (eq:initial_guess): "wet" means zeta + zb > 0 at
    some rule node; the lift is ``-max zb + eps0``.
  * Degree adaptation (eq:criteria_p): decided at the start of every step
    from h(zeta^n) on the rule nodes; mu_K >= h_lim keeps degree r.  A cell
    going from r to 0 is remapped conservatively: zeta-bar solves
    Hbar(zeta-bar) = Hbar(zeta^n), q-bar is the cell mean, c-bar = int(hc)/Hbar.
  * Tracer in a dry cell keeps its start-of-step value.  A cell counts as dry
    when Hbar <= 64 u |z_max| |K| (u = 2^-52, z_max the cell's largest depth
    sample): zero up to the round-off water that the scalar solve of
    Hbar = 0 leaves, where zeta + z_b cancels to a few ulps of |z_max| at the
    deepest nodes.
  * Tracer numerical diffusion (eq:numdiff) is the volume term as printed,
    - int nu h grad c . grad psi_i with the plain depth, on the sample rule,
    with nu_K = C |K| r^-2 S; the characteristic strain rate S of the
    resolved flow, which the paper does not define, is a given constant of
    the run.  A first-order decay, the reaction phi(c) = -kappa c of eq:shw,
    enters R as - kappa int h c psi_i (explicit, as eq:imex_shw takes the
    reactions).
  * Reactions that couple tracers (step_coupled) are the linear
    phi_k = sum_j B_kj c_j: R_k of every stage gets sum_j B_kj int h c_j psi_i
    of that stage's state on the volume rule, for every tracer before any
    takes the next stage.  The paper leaves the reaction terms' full
    discretisation open and names no rates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

DT = torch.float64
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
OPPOSITE = {WEST: EAST, EAST: WEST, SOUTH: NORTH, NORTH: SOUTH}
NORMAL = {WEST: (-1.0, 0.0), EAST: (1.0, 0.0), SOUTH: (0.0, -1.0), NORTH: (0.0, 1.0)}
BC_WALL, BC_ELEV, BC_OPEN, BC_PERIODIC = "wall", "elev", "open", "periodic"
BC_STATE, BC_DISCHARGE = "state", "discharge"


# ---------------------------------------------------------------------------
# Reference tables: basis nodes, quadrature rules, Lagrange basis (Sec. 3.2)
# ---------------------------------------------------------------------------

def gll_rule(n: int):
    """n-point Gauss-Legendre-Lobatto rule mapped to [0, 1].

    Nodes: -1, 1 and the roots of P'_{n-1}; weights 2 / (n (n-1) P_{n-1}(x)^2)
    on [-1, 1] (halved on [0, 1]).  Used for the basis support points
    (Sec. 3.2) and as a sub-grid rule family.
    """
    if n < 2:
        raise ValueError("GLL needs at least 2 points")
    leg = np.polynomial.legendre
    c = np.zeros(n)
    c[n - 1] = 1.0                      # P_{n-1}
    dc = leg.legder(c)                  # P'_{n-1}
    ddc = leg.legder(dc)
    if n > 2:
        x = np.sort(np.real(leg.legroots(dc)))
        for _ in range(3):              # polish the roots with Newton steps
            x = x - leg.legval(x, dc) / leg.legval(x, ddc)
        x = np.concatenate([[-1.0], x, [1.0]])
    else:
        x = np.array([-1.0, 1.0])
    w = 2.0 / (n * (n - 1) * leg.legval(x, c) ** 2)
    return (x + 1.0) / 2.0, w / 2.0


def gl_rule(n: int):
    """n-point Gauss-Legendre rule mapped to [0, 1] (Table 1, discharge mass)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


def eq_rule(n: int):
    """Closed equispaced rule on [0, 1]: composite trapezoid on n nodes.

    The paper's outlook suggests equispaced rules with many nodes (Sec. 6);
    the endpoint weight 1/(2(n-1)) enters the positivity bound.
    """
    if n < 2:
        raise ValueError("equispaced closed rule needs at least 2 points")
    x = np.arange(n, dtype=np.float64) / (n - 1)
    w = np.full(n, 1.0 / (n - 1))
    w[0] = w[-1] = 0.5 / (n - 1)
    return x, w


def rule_for(kind: str, n: int):
    if kind == "eq":
        return eq_rule(n)
    if kind == "gll":
        return gll_rule(n)
    raise ValueError(f"unknown rule {kind!r}")


def basis_nodes(r: int):
    """Support points of the degree-r nodal basis: (r+1)-point GLL (Sec. 3.2)."""
    return gll_rule(r + 1)[0]


def lagrange_values(nodes, x):
    """l_j(x) for the Lagrange polynomials on ``nodes``; shape [len(x), len(nodes)]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    out = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange_derivs(nodes, x):
    """l_j'(x), from the product rule applied to the Lagrange product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    out = np.zeros((len(x), n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term = term * (x - nodes[m]) / (nodes[j] - nodes[m])
            out[:, j] += term
    return out


def tensor_basis(r: int, X, Y):
    """psi_j(X, Y) = l_jx(X) l_jy(Y), j = jy*(r+1) + jx, and its reference gradient."""
    nodes = basis_nodes(r)
    lx, ly = lagrange_values(nodes, X), lagrange_values(nodes, Y)
    dlx, dly = lagrange_derivs(nodes, X), lagrange_derivs(nodes, Y)
    n1 = r + 1
    v = np.einsum("py,px->pyx", ly, lx).reshape(len(X), n1 * n1)
    gx = np.einsum("py,px->pyx", ly, dlx).reshape(len(X), n1 * n1)
    gy = np.einsum("py,px->pyx", dly, lx).reshape(len(X), n1 * n1)
    return v, gx, gy


# ---------------------------------------------------------------------------
# Runge-Kutta tableaux in Butcher form (Sec. 3.1, Appendix A)
# ---------------------------------------------------------------------------

def tableau(name: str):
    """Explicit Butcher tableau (A, b, c) as Python floats."""
    if name == "fe":                   # forward Euler, Prop. 3.2
        return [[0.0]], [1.0], [0.0]
    if name == "ssp3":                 # Table "SSP3" (Appendix A)
        A = [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.0]]
        return A, [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0], [0.0, 1.0, 0.5]
    if name in ("rk32", "imex"):       # explicit companion of the IMEX pair (Appendix A)
        chi = 1.0 - math.sqrt(2.0) / 2.0
        a32 = 0.5
        A = [[0.0, 0.0, 0.0], [2.0 * chi, 0.0, 0.0], [1.0 - a32, a32, 0.0]]
        b2 = (1.0 - 2.0 * chi) / (4.0 * chi)
        b = [1.0 - b2 - chi, b2, chi]
        return A, b, [0.0, 2.0 * chi, 1.0]
    if name == "rk44":                 # classical RK4 (Appendix A)
        A = [[0.0] * 4, [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]]
        return A, [1 / 6, 2 / 6, 2 / 6, 1 / 6], [0.0, 0.5, 0.5, 1.0]
    raise ValueError(f"unknown tableau {name!r}")


def implicit_tableau(name: str):
    """Implicit (DIRK) companion (A~, b~) of an IMEX pair: TR-BDF2 with
    chi = 1 - sqrt(2)/2 for "imex" (Appendix A, right tableau), so that
    b~ = b and c~ = c; None for the explicit schemes."""
    if name != "imex":
        return None
    chi = 1.0 - math.sqrt(2.0) / 2.0
    b2 = (1.0 - 2.0 * chi) / (4.0 * chi)
    b = [1.0 - b2 - chi, b2, chi]
    At = [[0.0, 0.0, 0.0], [chi, chi, 0.0], list(b)]
    return At, b


# ---------------------------------------------------------------------------
# Mesh: axis-aligned quadtree over an nx0 x ny0 grid of square coarse cells
# ---------------------------------------------------------------------------

class Mesh:
    """Quadtree leaves (level, i, j); cell = [x0+i*dx_L, x0+(i+1)*dx_L] x [...].

    dx_L = dx0 / 2**level.  ``bc`` = (west, east, south, north) boundary kinds.
    Faces (Sec. 3.2): a conforming interior face joins two equal cells; a
    hanging sub-face joins a fine cell to half of a coarse cell's side (2:1
    non-conforming meshes, Sec. 3.3 'Degree and h-adaptivity').
    """

    def __init__(self, nx0, ny0, x0, y0, dx0, level, ii, jj, bc=(BC_WALL,) * 4):
        self.nx0, self.ny0, self.x0, self.y0, self.dx0 = int(nx0), int(ny0), float(x0), float(y0), float(dx0)
        self.level = np.asarray(level, dtype=np.int64)
        self.ii = np.asarray(ii, dtype=np.int64)
        self.jj = np.asarray(jj, dtype=np.int64)
        self.bc = tuple(bc)
        self.K = len(self.level)
        if (self.bc[0] == BC_PERIODIC) != (self.bc[1] == BC_PERIODIC) or \
           (self.bc[2] == BC_PERIODIC) != (self.bc[3] == BC_PERIODIC):
            raise ValueError("periodic boundaries must come in pairs")
        self.dx = self.dx0 / (2.0 ** self.level)
        self.xc = self.x0 + self.ii * self.dx           # lower-left corner
        self.yc = self.y0 + self.jj * self.dx
        self._build()

    @staticmethod
    def uniform(nx, ny, x0, y0, dx, bc=(BC_WALL,) * 4):
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        return Mesh(nx, ny, x0, y0, dx, np.zeros(nx * ny, np.int64), ii.ravel(), jj.ravel(), bc)

    def _build(self):
        leaf = {}
        for k in range(self.K):
            key = (int(self.level[k]), int(self.ii[k]), int(self.jj[k]))
            if key in leaf:
                raise ValueError(f"duplicate cell {key}")
            leaf[key] = k
        area = float(np.sum(self.dx ** 2))
        if abs(area - self.nx0 * self.ny0 * self.dx0 ** 2) > 1e-9 * area:
            raise ValueError("cells do not tile the domain")
        per_x = self.bc[0] == BC_PERIODIC
        per_y = self.bc[2] == BC_PERIODIC
        step = {WEST: (-1, 0), EAST: (1, 0), SOUTH: (0, -1), NORTH: (0, 1)}
        faces, bfaces = [], []
        for k in range(self.K):
            L, i, j = int(self.level[k]), int(self.ii[k]), int(self.jj[k])
            nxL, nyL = self.nx0 << L, self.ny0 << L
            if not (0 <= i < nxL and 0 <= j < nyL):
                raise ValueError("cell outside the domain")
            for side in (WEST, EAST, SOUTH, NORTH):
                di, dj = step[side]
                ni, nj = i + di, j + dj
                if not (0 <= ni < nxL):
                    if per_x:
                        ni %= nxL
                    else:
                        bfaces.append((k, side))
                        continue
                if not (0 <= nj < nyL):
                    if per_y:
                        nj %= nyL
                    else:
                        bfaces.append((k, side))
                        continue
                if (L, ni, nj) in leaf:
                    if side in (EAST, NORTH):
                        faces.append((k, side, leaf[(L, ni, nj)], OPPOSITE[side], -1))
                    continue
                if L > 0 and (L - 1, ni >> 1, nj >> 1) in leaf:
                    sub = (j & 1) if side in (WEST, EAST) else (i & 1)
                    faces.append((k, side, leaf[(L - 1, ni >> 1, nj >> 1)], OPPOSITE[side], sub))
                    continue
                # the neighbour is finer: both children along this side must be leaves
                if side in (WEST, EAST):
                    kids = [(L + 1, 2 * ni + (1 if side == WEST else 0), 2 * nj + t) for t in (0, 1)]
                else:
                    kids = [(L + 1, 2 * ni + t, 2 * nj + (1 if side == SOUTH else 0)) for t in (0, 1)]
                if not all(kd in leaf for kd in kids):
                    raise ValueError(f"mesh is not 2:1 balanced at cell {k} side {side}")
        self.faces = faces        # (cellA, sideA, cellB, sideB, sub): A fine or equal
        self.bfaces = bfaces      # (cell, side)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

@dataclass
class Params:
    r: int = 1
    S: tuple = (8,)              # sub-grid nodes per direction, per level
    rule: str = "eq"             # "eq" (closed equispaced) or "gll"
    rk: str = "ssp3"
    g: float = 9.81
    eps: float = 0.1             # velocity desingularisation (eq:velocity)
    h_lim: float = 0.1           # degree-coarsening threshold (eq:criteria_p)
    eps0: float = 1e-8           # dry-cell lift (eq:initial_guess)
    newton_max: int = 20
    cfl: float = 0.2
    cfl_mode: int = 0            # 0: dt = cfl*min J/(lam l); 1: dt = cfl*min w1 J/(lam l)
    tracer: bool = False
    # tracer numerical diffusion (eq:numdiff): nu_K = C |K| r^-2 S with the
    # constant C and a characteristic strain rate S of the resolved flow (1/s)
    tracer_diff: float = 0.0
    tracer_strain: float = 0.0
    # first-order decay of the tracer, the reaction phi(c) = -kappa c of eq:shw (1/s)
    tracer_decay: float = 0.0
    tide: tuple = (0.0, 1.0, 0.0, 0.0)   # amplitude, period, phase, inflow tracer
    adapt_degree: bool = True
    # "subgrid": the S x S sample rule serves every element integral;
    # "paper": the rules of Table 1 (volume terms GL (floor(3r/2)+1)^2 with
    # samples of their own, faces and the continuity / tracer mass GLL
    # (r+2)^2, discharge mass GL (r+1)^2); S must then be r + 2 with rule "gll"
    quadrature: str = "subgrid"


@dataclass
class _Level:
    L: int
    S: int
    dx: float
    idx: torch.Tensor            # global cell indices of this level
    W: torch.Tensor              # [S*S] physical node weights dx^2 w_a w_b
    Bv: torch.Tensor             # [S*S, n_p] psi_j at node q = b*S + a
    Bx: torch.Tensor             # reference d/dxi psi_j
    By: torch.Tensor
    w1: float                    # endpoint weight of the 1-D rule
    zb: torch.Tensor = None      # [K_L, S*S] bathymetry depth samples
    pos: dict = field(default_factory=dict)


class _Vol:
    """Attribute view of a level's volume-rule tables (the paper's quadrature)."""

    def __init__(self, d):
        self.W, self.Bv, self.Bx, self.By = d["W"], d["Bv"], d["Bx"], d["By"]


def _pos(x):
    """max(x, 0) with the land-sea-mask convention: derivative 1 iff x > 0 (eq:mask)."""
    return torch.where(x > 0, x, torch.zeros_like(x))


def _inv_des(h, eps):
    """1/h_des = sqrt(2) h / sqrt(max(h^4, eps^4) + h^4) (eq:velocity)."""
    h4 = h ** 4
    return math.sqrt(2.0) * h / torch.sqrt(torch.clamp(h4, min=eps ** 4) + h4)


def _minimum(a, b):
    """min with ties resolved to the first argument."""
    return torch.where(a <= b, a, b)


def _maximum(a, b):
    return torch.where(a >= b, a, b)


def _safe_norm(x, y):
    n2 = x * x + y * y
    return torch.where(n2 > 0, torch.sqrt(torch.where(n2 > 0, n2, torch.ones_like(n2))), torch.zeros_like(n2))


# ---------------------------------------------------------------------------
# The oracle
# ---------------------------------------------------------------------------

class Oracle:
    def __init__(self, mesh: Mesh, p: Params):
        self.m, self.p = mesh, p
        r = p.r
        if r < 1:
            raise ValueError("r >= 1")
        self.n1 = r + 1
        self.np_ = (r + 1) ** 2
        K = mesh.K
        nlev = int(mesh.level.max()) + 1 if K else 1
        if len(p.S) < nlev:
            raise ValueError("need one S per level")
        self.levels = []
        self.cell_level_pos = torch.zeros(K, dtype=torch.long)
        for L in range(nlev):
            idx = np.nonzero(mesh.level == L)[0]
            if len(idx) == 0:
                continue
            S = int(p.S[L])
            if S < r + 2:
                raise ValueError("S must be >= r+2")
            xh, wh = rule_for(p.rule, S)
            X = np.tile(xh, S)                 # q = b*S + a  ->  x = xh[a]
            Y = np.repeat(xh, S)
            v, gx, gy = tensor_basis(r, X, Y)
            dx = mesh.dx0 / 2.0 ** L
            W = np.outer(wh, wh).ravel() * dx * dx   # W[b*S+a] = w_b w_a dx^2
            lv = _Level(L, S, dx, torch.as_tensor(idx, dtype=torch.long), torch.as_tensor(W),
                        torch.as_tensor(v), torch.as_tensor(gx), torch.as_tensor(gy), float(wh[0]))
            lv.zb = torch.zeros(len(idx), S * S, dtype=DT)
            lv.xh = xh
            lv.vol = None
            if p.quadrature == "paper":
                if p.rule != "gll" or S != r + 2:
                    raise ValueError("the paper's quadrature takes the GLL rule with S = r + 2 (Table 1)")
                nv = (3 * r) // 2 + 1
                xv, wv = gl_rule(nv)
                vv, gxv, gyv = tensor_basis(r, np.tile(xv, nv), np.repeat(xv, nv))
                lv.vol = dict(n=nv, xh=xv, W=torch.as_tensor(np.outer(wv, wv).ravel() * dx * dx),
                              Bv=torch.as_tensor(vv), Bx=torch.as_tensor(gxv), By=torch.as_tensor(gyv),
                              zb=torch.zeros(len(idx), nv * nv, dtype=DT))
            elif p.quadrature != "subgrid":
                raise ValueError(f"unknown quadrature {p.quadrature!r}")
            self.cell_level_pos[lv.idx] = torch.arange(len(idx))
            self.levels.append(lv)
        self.level_of = {lv.L: lv for lv in self.levels}
        # exact discharge mass matrix on the reference square (Table 1: GL (r+1)^2)
        xg, wg = gl_rule(r + 1)
        vg, _, _ = tensor_basis(r, np.tile(xg, r + 1), np.repeat(xg, r + 1))
        wgg = np.outer(wg, wg).ravel()
        self.Mq_ref = torch.as_tensor(vg.T @ (wgg[:, None] * vg))
        self.mean_w = torch.as_tensor(vg.T @ wgg)     # int psi_j over the reference cell
        self.nman = torch.zeros(K, dtype=DT)
        self.dbed = torch.zeros(K, dtype=DT)          # per-cell bed-elevation offset
        self.flag = torch.full((K,), r, dtype=torch.long)
        self.t = 0.0
        zero = torch.zeros(K, self.np_, dtype=DT)
        self.state = [zero.clone(), zero.clone(), zero.clone(), zero.clone()]
        self._build_faces()

    # -- geometry ----------------------------------------------------------
    def node_coords(self):
        """Sample-node coordinates, cell by cell, nodes q = b*S + a: x = x0 + (i + xh_a) dx.
        With the paper's quadrature the volume rule's nodes of every cell follow,
        cell by cell, in the same layout."""
        out = []
        m = self.m
        sets = [("xh", "S")] + ([("vol", None)] if self.p.quadrature == "paper" else [])
        for which, _ in sets:
            for k in range(m.K):
                lv = self.level_of[int(m.level[k])]
                xh, S = (lv.xh, lv.S) if which == "xh" else (lv.vol["xh"], lv.vol["n"])
                X = m.x0 + (m.ii[k] + np.tile(xh, S)) * lv.dx
                Y = m.y0 + (m.jj[k] + np.repeat(xh, S)) * lv.dx
                out.append(np.stack([X, Y], 1))
        return np.concatenate(out, 0) if out else np.zeros((0, 2))

    def dof_coords(self):
        """Basis support-point coordinates per cell, j = jy*(r+1)+jx."""
        m = self.m
        xi = basis_nodes(self.p.r)
        X = np.tile(xi, self.n1)
        Y = np.repeat(xi, self.n1)
        xs = m.x0 + (m.ii[:, None] + X[None, :]) * m.dx[:, None]
        ys = m.y0 + (m.jj[:, None] + Y[None, :]) * m.dx[:, None]
        return np.stack([xs, ys], -1)

    def set_bathymetry(self, b_flat):
        """b_flat: bed ELEVATION at node_coords(); stored as depth zb = -b."""
        b = torch.as_tensor(np.asarray(b_flat, dtype=np.float64))
        off = 0
        per_cell = []
        for k in range(self.m.K):
            S = self.level_of[int(self.m.level[k])].S
            per_cell.append((off, S))
            off += S * S
        voff = off
        if self.p.quadrature == "paper":
            for k in range(self.m.K):
                n = self.level_of[int(self.m.level[k])].vol["n"]
                per_cell[k] = per_cell[k] + (off, n)
                off += n * n
        if off != b.numel():
            raise ValueError("bathymetry size mismatch")
        for lv in self.levels:
            rows = [b[per_cell[k][0]: per_cell[k][0] + lv.S ** 2] for k in lv.idx.tolist()]
            lv.zb = -torch.stack(rows, 0) if rows else torch.zeros(0, lv.S ** 2, dtype=DT)
            if lv.vol is not None:
                n = lv.vol["n"]
                rows = [b[per_cell[k][2]: per_cell[k][2] + n * n] for k in lv.idx.tolist()]
                lv.vol["zb"] = -torch.stack(rows, 0) if rows else torch.zeros(0, n * n, dtype=DT)
        del voff

    def set_manning(self, n_cell):
        self.nman = torch.as_tensor(np.asarray(n_cell, dtype=np.float64)).clone()

    def set_bed_offset(self, db):
        self.dbed = torch.as_tensor(np.asarray(db, dtype=np.float64)).clone()

    def set_state(self, eta, qx, qy, c=None):
        K = self.m.K
        f = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64)).reshape(K, self.np_).clone()
        self.state = [f(eta), f(qx), f(qy), f(c) if c is not None else torch.zeros(K, self.np_, dtype=DT)]
        self.flag = torch.full((K,), self.p.r, dtype=torch.long)

    def get_state(self):
        return [s.clone().numpy() for s in self.state]

    def zb_eff(self, lv, dbed=None):
        """Depth samples of a level with the per-cell offset: b -> b + db, zb -> zb - db."""
        db = self.dbed if dbed is None else dbed
        return lv.zb - db[lv.idx][:, None]

    def zb_vol_eff(self, lv, dbed=None):
        """The same at the nodes of the paper's volume rule."""
        db = self.dbed if dbed is None else dbed
        return lv.vol["zb"] - db[lv.idx][:, None]

    def init_lake_at_rest(self, eta_nodal):
        """Definition 3.1: zeta_j = given value if some rule node is wet, else -max_q zb."""
        eta = torch.as_tensor(np.asarray(eta_nodal, dtype=np.float64)).reshape(self.m.K, self.np_).clone()
        for lv in self.levels:
            z = eta[lv.idx]
            zq = z @ lv.Bv.T
            zb = self.zb_eff(lv)
            wet = ((zq + zb) > 0).any(1)
            dry_val = -zb.max(1).values
            eta[lv.idx] = torch.where(wet[:, None], z, dry_val[:, None].expand_as(z))
        K = self.m.K
        self.set_state(eta, np.zeros((K, self.np_)), np.zeros((K, self.np_)), self.state[3].numpy())

    # -- faces -------------------------------------------------------------
    def _face_points(self, side, s):
        s = np.asarray(s, dtype=np.float64)
        if side == WEST:
            return np.zeros_like(s), s
        if side == EAST:
            return np.ones_like(s), s
        if side == SOUTH:
            return s, np.zeros_like(s)
        return s, np.ones_like(s)

    def _row_nodes(self, side, S):
        a = np.arange(S)
        if side == WEST:
            return a * S
        if side == EAST:
            return a * S + (S - 1)
        if side == SOUTH:
            return a
        return (S - 1) * S + a

    def _build_faces(self):
        m, r = self.m, self.p.r
        groups = {}
        for (kA, sA, kB, sB, sub) in m.faces:
            LA, LB = int(m.level[kA]), int(m.level[kB])
            key = (sA, sB, sub, LA, LB)
            groups.setdefault(key, []).append((kA, kB))
        self.face_groups = []
        for (sA, sB, sub, LA, LB), lst in groups.items():
            lvA, lvB = self.level_of[LA], self.level_of[LB]
            S = lvA.S
            s = lvA.xh
            XA, YA = self._face_points(sA, s)
            sBp = s if sub < 0 else (sub + s) / 2.0
            XB, YB = self._face_points(sB, sBp)
            vA, _, _ = tensor_basis(r, XA, YA)
            vB, _, _ = tensor_basis(r, XB, YB)
            _, wh = rule_for(self.p.rule, S)
            kA = torch.as_tensor([a for a, _ in lst], dtype=torch.long)
            kB = torch.as_tensor([b for _, b in lst], dtype=torch.long)
            self.face_groups.append(dict(
                sideA=sA, sideB=sB, sub=sub, lvA=lvA, lvB=lvB, kA=kA, kB=kB,
                posA=self.cell_level_pos[kA], posB=self.cell_level_pos[kB],
                rowA=torch.as_tensor(self._row_nodes(sA, S)),
                rowB=torch.as_tensor(self._row_nodes(sB, S)) if sub < 0 else None,
                vA=torch.as_tensor(vA), vB=torch.as_tensor(vB),
                wl=torch.as_tensor(wh) * lvA.dx, normal=NORMAL[sA]))
        bgroups = {}
        for (k, side) in m.bfaces:
            bgroups.setdefault((side, int(m.level[k])), []).append(k)
        self.bface_groups = []
        for (side, L), lst in bgroups.items():
            lv = self.level_of[L]
            X, Y = self._face_points(side, lv.xh)
            v, _, _ = tensor_basis(r, X, Y)
            _, wh = rule_for(self.p.rule, lv.S)
            k = torch.as_tensor(lst, dtype=torch.long)
            kind = m.bc[side]
            xs = m.x0 + (m.ii[lst][:, None] + X[None, :]) * lv.dx
            ys = m.y0 + (m.jj[lst][:, None] + Y[None, :]) * lv.dx
            self.bface_groups.append(dict(side=side, lv=lv, k=k, pos=self.cell_level_pos[k], xy=(xs, ys),
                                          row=torch.as_tensor(self._row_nodes(side, lv.S)),
                                          v=torch.as_tensor(v), wl=torch.as_tensor(wh) * lv.dx,
                                          normal=NORMAL[side], kind=kind))

    # -- the spatial operator ---------------------------------------------
    def residual(self, state, t, dbed=None, nman=None, friction=True):
        """Weak residuals F (eq:mass_rhs), G = (Gx, Gy) (eq:discharge_rhs plus the
        explicit friction L of eq:discharge_rhs_implicit; without it when
        friction=False) and R (eq:r_concentration, plus the numerical
        diffusion of eq:numdiff and the decay source -kappa int h c psi_i when
        they are set), for every degree-r test function, before any mass solve.

        Also returns the positivity time-step bound min over face nodes and
        face sides of w * J_K / (lambda l_Gamma) (Prop. 3.2, eq:deltat_fe),
        with w = the rule's endpoint weight (cfl_mode 1) or 1 (cfl_mode 0).
        """
        p = self.p
        g = p.g
        zeta, qx, qy, c = state
        nman = self.nman if nman is None else nman
        F = torch.zeros_like(zeta)
        Gx = torch.zeros_like(zeta)
        Gy = torch.zeros_like(zeta)
        R = torch.zeros_like(zeta)
        # ---- volume terms ----
        for lv in self.levels:
            idx = lv.idx
            if len(idx) == 0:
                continue
            Z, QX, QY, C = zeta[idx], qx[idx], qy[idx], c[idx]
            # the volume rule: the sample rule, or Table 1's GL rule
            vr = lv if lv.vol is None else _Vol(lv.vol)
            zq = Z @ vr.Bv.T
            zx = (Z @ vr.Bx.T) / lv.dx
            zy = (Z @ vr.By.T) / lv.dx
            qxq, qyq, cq = QX @ vr.Bv.T, QY @ vr.Bv.T, C @ vr.Bv.T
            zbv = self.zb_eff(lv, dbed) if lv.vol is None else self.zb_vol_eff(lv, dbed)
            h = _pos(zq + zbv)
            ih = _inv_des(h, p.eps)
            ux, uy = qxq * ih, qyq * ih
            gam = g * nman[idx][:, None] ** 2 * _safe_norm(qxq, qyq) * ih ** (7.0 / 3.0)
            W = vr.W
            Bx, By, Bv = vr.Bx / lv.dx, vr.By / lv.dx, vr.Bv
            # F_i += int q . grad psi_i
            F = F.index_add(0, idx, (W * qxq) @ Bx + (W * qyq) @ By)
            # G_i,k += int q_k (u . grad psi_i) - g h d_k zeta psi_i - gamma q_k psi_i
            fr = 1.0 if friction else 0.0
            Gx = Gx.index_add(0, idx, (W * qxq * ux) @ Bx + (W * qxq * uy) @ By
                              - (W * g * h * zx) @ Bv - fr * ((W * gam * qxq) @ Bv))
            Gy = Gy.index_add(0, idx, (W * qyq * ux) @ Bx + (W * qyq * uy) @ By
                              - (W * g * h * zy) @ Bv - fr * ((W * gam * qyq) @ Bv))
            if p.tracer:
                R = R.index_add(0, idx, (W * cq * qxq) @ Bx + (W * cq * qyq) @ By)
                nu = p.tracer_diff * lv.dx ** 2 * p.tracer_strain / p.r ** 2
                if nu != 0.0:
                    # eq:numdiff: - int nu h grad c . grad psi_i
                    cx, cy = (C @ vr.Bx.T) / lv.dx, (C @ vr.By.T) / lv.dx
                    R = R.index_add(0, idx, -((W * nu * h * cx) @ Bx + (W * nu * h * cy) @ By))
                if p.tracer_decay != 0.0:
                    # the reaction source int h phi(c) psi_i with phi(c) = -kappa c
                    R = R.index_add(0, idx, -((W * p.tracer_decay * h * cq) @ Bv))
        dtb = torch.tensor(float("inf"), dtype=DT)
        # ---- interior faces ----
        for fg in self.face_groups:
            kA, kB = fg["kA"], fg["kB"]
            vA, vB = fg["vA"], fg["vB"]
            nx, ny = fg["normal"]
            lvA, lvB = fg["lvA"], fg["lvB"]
            zbA = self.zb_eff(lvA, dbed)[fg["posA"]][:, fg["rowA"]]
            if fg["sub"] < 0:
                zbB = self.zb_eff(lvB, dbed)[fg["posB"]][:, fg["rowB"]]
            else:
                # the coarse side's bed at a hanging node is the sample taken at the
                # same point by the fine side, with the coarse cell's own offset
                db = self.dbed if dbed is None else dbed
                zbB = self.zb_eff(lvA, dbed)[fg["posA"]][:, fg["rowA"]] + db[kA][:, None] - db[kB][:, None]
            trA = [s[kA] @ vA.T for s in state]
            trB = [s[kB] @ vB.T for s in state]
            fl = self._flux(trA, trB, zbA, zbB, nx, ny)
            wl = fg["wl"]
            self_contrib = lambda f, v: (wl * f) @ v
            F = F.index_add(0, kA, -self_contrib(fl["mass"], vA))
            F = F.index_add(0, kB, self_contrib(fl["mass"], vB))
            Gx = Gx.index_add(0, kA, -self_contrib(fl["momx"], vA) + self_contrib(fl["presx"], vA))
            Gx = Gx.index_add(0, kB, self_contrib(fl["momx"], vB) + self_contrib(fl["presx"], vB))
            Gy = Gy.index_add(0, kA, -self_contrib(fl["momy"], vA) + self_contrib(fl["presy"], vA))
            Gy = Gy.index_add(0, kB, self_contrib(fl["momy"], vB) + self_contrib(fl["presy"], vB))
            if p.tracer:
                R = R.index_add(0, kA, -self_contrib(fl["trac"], vA))
                R = R.index_add(0, kB, self_contrib(fl["trac"], vB))
            lam = fl["lam"]
            l = lvA.dx
            for lv in (lvA, lvB):
                w = lv.w1 if p.cfl_mode == 1 else 1.0
                bnd = torch.where(lam > 0, w * lv.dx ** 2 / (lam * l + (lam <= 0)), torch.full_like(lam, float("inf")))
                if bnd.numel():
                    dtb = torch.minimum(dtb, bnd.min())
        # ---- boundary faces (ghost states) ----
        for bg in self.bface_groups:
            k, v = bg["k"], bg["v"]
            nx, ny = bg["normal"]
            lv = bg["lv"]
            zbA = self.zb_eff(lv, dbed)[bg["pos"]][:, bg["row"]]
            trA = [s[k] @ v.T for s in state]
            trB = self._ghost(bg["kind"], trA, nx, ny, t, bg.get("given"))
            fl = self._flux(trA, trB, zbA, zbA, nx, ny)
            wl = bg["wl"]
            F = F.index_add(0, k, -(wl * fl["mass"]) @ v)
            Gx = Gx.index_add(0, k, -(wl * fl["momx"]) @ v + (wl * fl["presx"]) @ v)
            Gy = Gy.index_add(0, k, -(wl * fl["momy"]) @ v + (wl * fl["presy"]) @ v)
            if p.tracer:
                R = R.index_add(0, k, -(wl * fl["trac"]) @ v)
            lam = fl["lam"]
            w = lv.w1 if p.cfl_mode == 1 else 1.0
            bnd = torch.where(lam > 0, w * lv.dx / (lam + (lam <= 0)), torch.full_like(lam, float("inf")))
            if bnd.numel():
                dtb = torch.minimum(dtb, bnd.min())
        return F, Gx, Gy, R, dtb

    def set_boundary_state(self, fn):
        """Boundary data of the state and discharge sides: fn(x, y) -> (zeta, qx,
        qy, c) at the face nodes (arrays of the shape of x)."""
        for bg in self.bface_groups:
            if bg["kind"] in (BC_STATE, BC_DISCHARGE):
                vals = fn(*bg["xy"])
                bg["given"] = [torch.as_tensor(np.broadcast_to(np.asarray(v, dtype=np.float64), bg["xy"][0].shape).copy())
                               for v in vals]

    def _ghost(self, kind, tr, nx, ny, t, given=None):
        zeta, qx, qy, c = tr
        if kind in (BC_STATE, BC_DISCHARGE) and given is None:
            raise ValueError("boundary data of a state or discharge side are not set")
        if kind == BC_STATE:
            return list(given)
        if kind == BC_DISCHARGE:
            inflow = (given[1] * nx + given[2] * ny) < 0
            return [zeta, given[1], given[2], torch.where(inflow, given[3], c)]
        if kind == BC_WALL:
            qn = qx * nx + qy * ny
            return [zeta, qx - 2.0 * qn * nx, qy - 2.0 * qn * ny, c]
        if kind == BC_OPEN:
            return [zeta, qx, qy, c]
        if kind == BC_ELEV:
            A, T, ph, cin = self.p.tide
            zb = torch.full_like(zeta, A * math.sin(2.0 * math.pi * t / T + ph))
            inflow = (qx * nx + qy * ny) < 0
            return [zb, qx, qy, torch.where(inflow, torch.full_like(c, cin), c)]
        raise ValueError(kind)

    def _flux(self, trA, trB, zbA, zbB, nx, ny):
        """Numerical fluxes at face nodes, seen from side A (normal n = outward of A).

        Rusanov speed (eq:lxf_parameter) with desingularised velocities
        (eq:velocity); hydrostatic reconstruction (eq:hydro_rec,
        eq:hydro_rec_vars) in every flux.  Side B receives the negated
        conservative fluxes and the same pressure term (eq:discharge_rhs).
        """
        g, eps = self.p.g, self.p.eps
        zA, qxA, qyA, cA = trA
        zB, qxB, qyB, cB = trB
        hA, hB = _pos(zA + zbA), _pos(zB + zbB)
        ihA, ihB = _inv_des(hA, eps), _inv_des(hB, eps)
        uxA, uyA, uxB, uyB = qxA * ihA, qyA * ihA, qxB * ihB, qyB * ihB
        unA = uxA * nx + uyA * ny
        unB = uxB * nx + uyB * ny
        lam = _maximum(torch.abs(unA) + torch.sqrt(g * hA), torch.abs(unB) + torch.sqrt(g * hB))
        zs = _minimum(zbA, zbB)                      # z*_b = min(zb-, zb+)
        hsA, hsB = _pos(zA + zs), _pos(zB + zs)      # h* = max(zeta + z*, 0)
        qsxA, qsyA, qsxB, qsyB = hsA * uxA, hsA * uyA, hsB * uxB, hsB * uyB   # q* = h* u
        esA, esB = _maximum(zA, -zs), _maximum(zB, -zs)                    # zeta* = max(zeta, -z*)
        mass = 0.5 * ((qsxA + qsxB) * nx + (qsyA + qsyB) * ny) + 0.5 * lam * (esA - esB)
        momx = 0.5 * (qsxA * unA + qsxB * unB) + 0.5 * lam * (qsxA - qsxB)
        momy = 0.5 * (qsyA * unA + qsyB * unB) + 0.5 * lam * (qsyA - qsyB)
        pres = 0.5 * g * 0.5 * (hsA + hsB) * (esA - esB)
        trac = 0.5 * ((qsxA * cA + qsxB * cB) * nx + (qsyA * cA + qsyB * cB) * ny) \
            + 0.5 * lam * (hsA * cA - hsB * cB)
        return dict(mass=mass, momx=momx, momy=momy, presx=pres * nx, presy=pres * ny, trac=trac, lam=lam)

    # -- per-cell mass terms and solves -------------------------------------
    def _depth_terms(self, lv, pos, zeta_nodal, dbed=None):
        """h at rule nodes, land-sea mask (eq:mask), H (eq:depth_rhs)."""
        zq = zeta_nodal @ lv.Bv.T
        s = zq + self.zb_eff(lv, dbed)[pos]
        h = _pos(s)
        mask = s > 0
        H = (lv.W * h) @ lv.Bv
        return h, mask, H

    @staticmethod
    def _chol_solve(A, rhs):
        """Batched Cholesky solve with the pivot test; returns (x, ok)."""
        if A.shape[0] == 0:
            return rhs.clone(), torch.ones(0, dtype=torch.bool)
        L, info = torch.linalg.cholesky_ex(A)
        tr = torch.diagonal(A, dim1=-2, dim2=-1).sum(-1)
        piv = torch.diagonal(L, dim1=-2, dim2=-1) ** 2
        ok = (info == 0) & (piv > 1e-14 * tr[:, None]).all(-1) & (tr > 0)
        x = torch.zeros_like(rhs)
        if ok.any():
            x_ok = torch.cholesky_solve(rhs[ok].unsqueeze(-1), L[ok]).squeeze(-1)
            x = x.index_put((ok.nonzero().squeeze(1),), x_ok)
        return x, ok

    def _newton(self, lv, pos, T, zeta_guess_nodal, full, dbed=None):
        """Element-wise Newton for H(zeta) = T (eq:newton, eq:mass_matrix).

        ``full``: bool per cell, True for degree-r cells (vector unknown),
        False for degree-0 cells (scalar unknown, mass = wet area).
        Returns the new nodal zeta, iteration counts and the final depths/H.
        """
        p = self.p
        npn = self.np_
        zb = self.zb_eff(lv, dbed)[pos]
        W, Bv = lv.W, lv.Bv
        # degree-0 cells: the target is the sum over the degree-r test functions
        Tbar = T.sum(1)
        z = zeta_guess_nodal.clone()
        # degree-0 unknown is the stored constant
        z = torch.where(full[:, None], z, z[:, :1].expand(-1, npn))
        # initial guess, eq:initial_guess
        zq = z @ Bv.T
        wet_any = ((zq + zb) > 0).any(1)
        lift = -zb.max(1).values + p.eps0
        z = torch.where(wet_any[:, None], z, lift[:, None].expand(-1, npn))
        k = z.shape[0]
        its = torch.zeros(k, dtype=torch.long)

        def terms(z):
            zq = torch.where(full[:, None], z @ Bv.T, z[:, :1].expand(-1, Bv.shape[0]))
            s = zq + zb
            h = _pos(s)
            mask = s > 0
            H = (W * h) @ Bv
            Hbar = (W * h).sum(1)
            Awet = (W * mask).sum(1)
            return h, mask, H, Hbar, Awet

        h, mask, H, Hbar, Awet = terms(z)
        active = Awet > 0
        fallback_used = torch.zeros(k, dtype=torch.bool)
        for _ in range(p.newton_max):
            if not bool(active.any()):
                break
            # degree-r: masked Jacobian M_ij = sum W psi_i psi_j l (eq:mass_matrix)
            M = torch.einsum("kq,qi,qj->kij", W * mask, Bv, Bv)
            dz_full, ok = self._chol_solve(M, H - T)
            # constant-mode update: degree-0 cells always, degree-r cells whose
            # masked matrix is numerically singular
            s_const = torch.where(Awet > 0, (Hbar - Tbar) / torch.where(Awet > 0, Awet, torch.ones_like(Awet)),
                                  torch.zeros_like(Awet))
            use_full = full & ok
            fallback_used |= active & full & ~ok
            dz = torch.where(use_full[:, None], dz_full, s_const[:, None].expand(-1, npn))
            dz = torch.where(active[:, None], dz, torch.zeros_like(dz))
            znew = z - dz
            its = its + active.long()
            hn, maskn, Hn, Hbarn, Awetn = terms(znew)
            l1 = torch.where(full, dz.abs().sum(1), dz[:, 0].abs())
            conv = (maskn == mask).all(1) | (l1 <= 1e-16)
            z, h, mask, H, Hbar, Awet = znew, hn, maskn, Hn, Hbarn, Awetn
            active = active & ~conv & (Awet > 0)
        return z, its, h, H, Hbar, fallback_used

    def _dry_floor(self, lv):
        """Round-off water of a dry cell: 64 u |z_max| |K| (u = 2^-52)."""
        return 64.0 * 2.0 ** -52 * self.zb_eff(lv).max(1).values.abs() * lv.dx ** 2

    def _tracer_solve(self, lv, h, CT, c_keep, full):
        """hc-mass system (eq:algebraic_concentration, eq:mass_matrix_concentration)."""
        W, Bv = lv.W, lv.Bv
        Hbar = (W * h).sum(1)
        wet = Hbar > self._dry_floor(lv)   # dry up to round-off water
        Hm = torch.einsum("kq,qi,qj->kij", W * h, Bv, Bv)
        x, ok = self._chol_solve(Hm, CT)
        # constant-mode fallback: c = c_keep + s with sum_i (Hm (c_keep + s))_i = sum CT
        Hc = torch.einsum("kij,kj->ki", Hm, c_keep).sum(1)
        safe = torch.where(wet, Hbar, torch.ones_like(Hbar))
        s = (CT.sum(1) - Hc) / safe
        fb = c_keep + s[:, None]
        cbar = CT.sum(1) / safe
        out = torch.where((full & ok)[:, None], x, fb)
        out = torch.where(full[:, None], out, cbar[:, None].expand_as(out))
        return torch.where(wet[:, None], out, c_keep)

    def _adapt(self, zeta, qx, qy, c, flag):
        """Degree decision at a step start (eq:criteria_p): r_K = 0 iff the
        smallest depth over the rule nodes is below h_lim; a cell going from r
        to 0 is remapped conservatively in place (zeta-bar solves
        Hbar(zeta-bar) = Hbar(zeta^n), q-bar is the cell mean, c-bar =
        int(h c)/Hbar).  Returns the new flags."""
        p = self.p
        r = p.r
        newflag = flag.clone()
        for lv in self.levels:
            pos = torch.arange(len(lv.idx))
            h, mask, H = self._depth_terms(lv, pos, zeta[lv.idx])
            mu = h.min(1).values
            nf = torch.where(mu >= p.h_lim, torch.full_like(mu, r, dtype=torch.long),
                             torch.zeros_like(mu, dtype=torch.long)) if p.adapt_degree else \
                torch.full((len(lv.idx),), r, dtype=torch.long)
            newflag[lv.idx] = nf
            remap = (flag[lv.idx] == r) & (nf == 0)
            if bool(remap.any()):
                ridx = lv.idx[remap]
                rpos = pos[remap]
                Hbar = (lv.W * h[remap]).sum(1)
                zmean = zeta[ridx] @ self.mean_w
                zguess = zmean[:, None].expand(-1, self.np_)
                Tn = torch.zeros(len(ridx), self.np_, dtype=DT)
                Tn[:, 0] = Hbar               # the scalar solve only sees the sum
                full0 = torch.zeros(len(ridx), dtype=torch.bool)
                znew, _, _, _, _, _ = self._newton(lv, rpos, Tn, zguess, full0)
                hc = (lv.W * h[remap] * (c[ridx] @ lv.Bv.T)).sum(1)
                cmean = c[ridx] @ self.mean_w
                wet = Hbar > self._dry_floor(lv)[remap]
                cbar = torch.where(wet, hc / torch.where(wet, Hbar, torch.ones_like(Hbar)), cmean)
                zeta[ridx] = znew[:, :1].expand(-1, self.np_)
                qx[ridx] = (qx[ridx] @ self.mean_w)[:, None].expand(-1, self.np_)
                qy[ridx] = (qy[ridx] @ self.mean_w)[:, None].expand(-1, self.np_)
                c[ridx] = cbar[:, None].expand(-1, self.np_)
        return newflag

    def adapted(self):
        """The state and degree flags as the next step sees them after its
        degree decision and remap (the oracle's own state is left unchanged):
        what a caller that fuses the next step's start into the end of a step
        holds."""
        st = [x.clone() for x in self.state]
        flag = self._adapt(st[0], st[1], st[2], st[3], self.flag)
        return [x.numpy() for x in st], flag.numpy()

    def adapted_state(self):
        return self.adapted()[0]

    # -- one time step ------------------------------------------------------
    def step(self, dt=None):
        """One explicit RK step in Butcher form (Sec. 3.1, eq:algebraic_elevation,
        eq:algebraic_discharge, eq:algebraic_concentration)."""
        gen = self.stepper(dt)
        while True:
            try:
                next(gen)
            except StopIteration as done:
                return done.value

    def stepper(self, dt=None):
        """The step of ``step`` taken stage by stage: after the residual of each
        stage state u^(l) it yields (l, u^(l), [F, Gx, Gy, R]) and resumes once
        the caller is done with them; a caller may add to R (the reaction
        source of eq:shw, explicit in every stage as in eq:imex_shw) before it
        resumes.  Returns the step's diagnostics."""
        p = self.p
        A, b, cc = tableau(p.rk)
        imp = implicit_tableau(p.rk)     # IMEX: friction with the DIRK companion
        s = len(b)
        zeta, qx, qy, c = [x.clone() for x in self.state]
        r = p.r
        K = self.m.K
        diag = dict(min_target=float("inf"), n_viol=0, newton_it=0, n_fallback=0)
        # ---- degree adaptation (eq:criteria_p) and conservative remap ----
        newflag = self._adapt(zeta, qx, qy, c, self.flag)
        self.flag = newflag
        full_all = newflag == r
        # ---- start-of-step quantities H^n, Q~^n, C~^n ----
        Hn = torch.zeros(K, self.np_, dtype=DT)
        Cn = torch.zeros(K, self.np_, dtype=DT)
        for lv in self.levels:
            pos = torch.arange(len(lv.idx))
            h, _, H = self._depth_terms(lv, pos, zeta[lv.idx])
            Hn[lv.idx] = H
            if p.tracer:
                Cn[lv.idx] = (lv.W * h * (c[lv.idx] @ lv.Bv.T)) @ lv.Bv
        Jac = torch.as_tensor(self.m.dx ** 2)
        Mq = self.Mq_ref[None] * Jac[:, None, None]
        Qxn = torch.einsum("kij,kj->ki", Mq, qx)
        Qyn = torch.einsum("kij,kj->ki", Mq, qy)
        state_n = [zeta, qx, qy, c]
        res = []
        lres = []                        # IMEX: implicit-part residuals L of each stage
        cur = state_n
        self.last_stages = [state_n]     # stage states u^(1) = u^n, u^(2), ..., then u^(n+1)
        t0 = self.t
        for l in range(s + 1):
            if l > 0:
                coef = A[l] if l < s else b
                upto = l if l < s else s
                acc = [None] * 4
                for m_ in range(upto):
                    a = coef[m_]
                    if a == 0.0:
                        continue
                    for f in range(4):
                        term = a * res[m_][f]
                        acc[f] = term if acc[f] is None else acc[f] + term
                acc = [x if x is not None else torch.zeros_like(Hn) for x in acc]
                T = Hn + dt * acc[0]
                QX = Qxn + dt * acc[1]
                QY = Qyn + dt * acc[2]
                if imp is not None:
                    # eq:algebraic_discharge: + dt sum_m a~_lm L^(m)
                    coeft = imp[0][l] if l < s else imp[1]
                    accL = [torch.zeros_like(Hn), torch.zeros_like(Hn)]
                    for m_ in range(upto):
                        if coeft[m_] != 0.0:
                            accL = [accL[0] + coeft[m_] * lres[m_][0], accL[1] + coeft[m_] * lres[m_][1]]
                    QX = QX + dt * accL[0]
                    QY = QY + dt * accL[1]
                CT = Cn + dt * acc[3]
                Tbar = T.sum(1)
                diag["min_target"] = min(diag["min_target"], float(Tbar.min()) if K else 0.0)
                diag["n_viol"] += int((Tbar < 0).sum())
                nz = torch.zeros_like(zeta)
                nc = torch.zeros_like(c)
                for lv in self.levels:
                    idx = lv.idx
                    pos = torch.arange(len(idx))
                    full = full_all[idx]
                    zl, its, h, _, _, fb = self._newton(lv, pos, T[idx], zeta[idx], full)
                    diag["newton_it"] = max(diag["newton_it"], int(its.max()) if len(its) else 0)
                    diag["n_fallback"] += int(fb.sum())
                    nz[idx] = zl
                    if p.tracer:
                        nc[idx] = self._tracer_solve(lv, h, CT[idx], c[idx], full)
                    else:
                        nc[idx] = c[idx]
                # discharge (eq:algebraic_discharge with A = exact mass matrix; for
                # an IMEX stage A^(l) = M + a~_ll dt Gam(q^(l-1), h^(l-1)),
                # eq:mass_matrix_discharge, the previous stage's friction)
                if imp is not None and l < s and imp[0][l][l] != 0.0:
                    _, _, Gam = self._friction(cur)
                    nqx, nqy, qfb = self._discharge_solve(Mq, Jac, Gam, imp[0][l][l] * dt, QX, QY, full_all)
                else:
                    nqx, nqy, qfb = self._discharge_solve(Mq, Jac, None, 0.0, QX, QY, full_all)
                diag["n_fallback"] += int(qfb.sum())
                cur = [nz, nqx, nqy, nc]
                self.last_stages.append(cur)
            if l < s:
                F, Gx, Gy, R, dtb = self.residual(cur, t0 + cc[l] * (dt if dt is not None else 0.0),
                                                  friction=imp is None)
                if imp is not None:
                    Lx, Ly, _ = self._friction(cur)
                    lres.append((Lx, Ly))
                if l == 0 and dt is None:
                    dt = p.cfl * float(dtb)
                    if l == 0 and cc[0] != 0.0:
                        raise ValueError("first stage must have c = 0")
                res.append([F, Gx, Gy, R])
                yield l, cur, res[l]
        self.state = cur
        self.t = t0 + dt
        mass = 0.0
        for lv in self.levels:
            h, _, _ = self._depth_terms(lv, torch.arange(len(lv.idx)), cur[0][lv.idx])
            mass += float((lv.W * h).sum())
        diag.update(dt=dt, mass=mass, n_r0=int((self.flag == 0).sum()))
        return diag

    def _discharge_solve(self, Mq, Jac, Gam, ct, QX, QY, full):
        """Discharge solve of a stage (eq:algebraic_discharge): A q = Q with A
        the exact mass matrix M times |K| (Table 1), or for an IMEX stage
        A = M + ct Gam (eq:mass_matrix_discharge, ct = a~_ll dt; Gam None: no
        implicit part).  A degree-0 cell takes the constant
        q = sum_i Q_i / (|K| + ct sum_ij Gam_ij), the same equation tested with
        the constant function.  The matrix is SPD; a Cholesky pivot below
        1e-14 trace (friction weights beyond the reach of double precision, at
        roundoff-thin nodes) gives that constant-mode update too.
        Returns (qx, qy, fallback) per cell."""
        if Gam is None:
            Amat, Asum = Mq, Jac
        else:
            Amat = Mq + ct * Gam
            Asum = Jac + ct * Gam.sum((1, 2))
        qxf, ok = self._chol_solve(Amat, QX)
        qyf, _ = self._chol_solve(Amat, QY)
        fb = full & ~ok
        use = (full & ok)[:, None]
        qx0 = (QX.sum(1) / Asum)[:, None].expand_as(qxf)
        qy0 = (QY.sum(1) / Asum)[:, None].expand_as(qyf)
        return torch.where(use, qxf, qx0), torch.where(use, qyf, qy0), fb

    def _friction(self, state, nman=None):
        """Implicit-part terms of the discharge equation at a state.

        L_i = -int gamma(|q|, h_des) q psi_i (eq:discharge_rhs_implicit: the
        desingularised depth of eq:velocity) and the matrix
        Gam_ij = int gamma(|q|, h) psi_i psi_j of eq:mass_matrix_discharge with
        the plain depth h, gamma(q, h) = g n^2 q / h^(7/3) (eq:manning), both on
        the sample rule.  At a dry node (h = 0) the friction coefficient of the
        matrix is taken as zero: the node carries no water column, so it adds
        nothing to the matrix (gamma q -> 0 there).  For h >= eps the two depths
        coincide (h_des = h)."""
        p = self.p
        zeta, qx, qy = state[0], state[1], state[2]
        nman = self.nman if nman is None else nman
        K = self.m.K
        Lx = torch.zeros(K, self.np_, dtype=DT)
        Ly = torch.zeros(K, self.np_, dtype=DT)
        Gam = torch.zeros(K, self.np_, self.np_, dtype=DT)
        for lv in self.levels:
            idx = lv.idx
            if len(idx) == 0:
                continue
            # the volume rule (with the paper's quadrature the friction matrix
            # takes it too: its depth needs bathymetry values at its nodes)
            vr = lv if lv.vol is None else _Vol(lv.vol)
            zq = zeta[idx] @ vr.Bv.T
            qxq, qyq = qx[idx] @ vr.Bv.T, qy[idx] @ vr.Bv.T
            zbv = self.zb_eff(lv, None) if lv.vol is None else self.zb_vol_eff(lv, None)
            h = _pos(zq + zbv)
            ih = _inv_des(h, p.eps)
            gn2q = p.g * nman[idx][:, None] ** 2 * _safe_norm(qxq, qyq)
            gam_des = gn2q * ih ** (7.0 / 3.0)                     # gamma(|q|, h_des)
            live = (h > 0) & (gn2q > 0)
            hs = torch.where(live, h, torch.ones_like(h))
            gam_h = torch.where(live, gn2q / hs ** (7.0 / 3.0), torch.zeros_like(h))   # gamma(|q|, h)
            W, Bv = vr.W, vr.Bv
            Lx[idx] = -((W * gam_des * qxq) @ Bv)
            Ly[idx] = -((W * gam_des * qyq) @ Bv)
            Gam[idx] = torch.einsum("kq,qi,qj->kij", W * gam_h, Bv, Bv)
        return Lx, Ly, Gam

    def hc_moments(self, state):
        """int h c psi_i over each cell on the volume rule (the rule of the
        residual's volume terms), with h the plain depth of the state's zeta:
        the source int h phi psi_i of eq:shw for phi = c."""
        zeta, c = state[0], state[3]
        S = torch.zeros_like(zeta)
        for lv in self.levels:
            idx = lv.idx
            if len(idx) == 0:
                continue
            vr = lv if lv.vol is None else _Vol(lv.vol)
            zbv = self.zb_eff(lv) if lv.vol is None else self.zb_vol_eff(lv)
            h = _pos(zeta[idx] @ vr.Bv.T + zbv)
            S[idx] = (vr.W * h * (c[idx] @ vr.Bv.T)) @ vr.Bv
        return S

    def apply_operator(self, state=None, t=None):
        st = self.state if state is None else [torch.as_tensor(np.asarray(s, dtype=np.float64)).reshape(self.m.K, self.np_) for s in state]
        F, Gx, Gy, R, dtb = self.residual(st, self.t if t is None else t)
        return F.numpy(), Gx.numpy(), Gy.numpy(), R.numpy(), float(dtb)

    def total_mass(self):
        mass = 0.0
        for lv in self.levels:
            h, _, _ = self._depth_terms(lv, torch.arange(len(lv.idx)), self.state[0][lv.idx])
            mass += float((lv.W * h).sum())
        return mass

    def conserved(self, state=None):
        """Per-dof depth and tracer-mass integrals H_i = int psi_i h and
        C_i = int psi_i h c (eq:depth_rhs, eq:concentration_rhs) of a state
        (default: the current one), and the cell means Hbar_K / |K|."""
        st = self.state if state is None else [torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(self.m.K, self.np_)
                                               for x in state]
        H = torch.zeros(self.m.K, self.np_, dtype=DT)
        C = torch.zeros(self.m.K, self.np_, dtype=DT)
        for lv in self.levels:
            pos = torch.arange(len(lv.idx))
            h, _, Hl = self._depth_terms(lv, pos, st[0][lv.idx])
            H[lv.idx] = Hl
            C[lv.idx] = (lv.W * h * (st[3][lv.idx] @ lv.Bv.T)) @ lv.Bv
        mean_depth = H.sum(1) / torch.as_tensor(self.m.dx ** 2)
        return H.numpy(), C.numpy(), mean_depth.numpy()

    def depth_integrals(self):
        """Per-cell Hbar_K and per-dof H_i at the current state."""
        Hn = torch.zeros(self.m.K, self.np_, dtype=DT)
        for lv in self.levels:
            _, _, H = self._depth_terms(lv, torch.arange(len(lv.idx)), self.state[0][lv.idx])
            Hn[lv.idx] = H
        return Hn.numpy()


def step_coupled(oracles, B, dt):
    """One step of M tracers c_1..c_M carried by one flow, with the linear
    reactions phi_k(c_1, ..., c_M) = sum_j B_kj c_j of eq:shw.

    Each tracer is an Oracle of its own whose flow is the same (same mesh,
    parameters, bathymetry and flow state), so their flows are identical.  The
    steps run stage by stage together: the reaction enters every stage
    explicitly, as eq:imex_shw takes it,

        h^(l) c_k^(l) = h^n c_k^n - dt sum_m a_lm (div(q c_k))^(m)
                        + dt sum_m a_lm h^(m) phi_k(c^(m)),

    so after the residuals of stage m each tracer's R gets
    sum_j B_kj int h^(m) c_j^(m) psi_i before any tracer takes stage m + 1.
    dt must be given.  Returns each tracer's step diagnostics.
    """
    B = np.asarray(B, dtype=np.float64)
    M = len(oracles)
    if B.shape != (M, M):
        raise ValueError("B must be M x M for M tracers")
    if dt is None or not dt > 0.0:
        raise ValueError("the coupled step needs a fixed dt > 0")
    gens = [o.stepper(dt) for o in oracles]
    diags = [None] * M
    while True:
        outs = []
        for k, g in enumerate(gens):
            try:
                outs.append(next(g))
            except StopIteration as done:
                diags[k] = done.value
        if not outs:
            return diags
        if len(outs) != M:
            raise RuntimeError("the tracers' steps have different numbers of stages")
        Sm = [o.hc_moments(cur) for o, (_, cur, _) in zip(oracles, outs)]
        for k, (_, _, res) in enumerate(outs):
            src = torch.zeros_like(res[3])
            for j in range(M):
                if B[k, j] != 0.0:
                    src = src + B[k, j] * Sm[j]
            res[3] = res[3] + src
