"""Thin ctypes binding of include/sw.h (argument marshalling only).

Device buffers are torch CUDA tensors; every step of the method runs in the
HIP library.  Loading fails loudly if libswdg.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libswdg.so")

BC = {"wall": 0, "elev": 1, "open": 2, "periodic": 3, "state": 4, "discharge": 5}
RULE = {"eq": 0, "gll": 1}
RK = {"fe": 0, "ssp3": 1, "rk32": 2, "rk44": 3, "imex": 4}
QUADRATURE = {"subgrid": 0, "paper": 1}

EXPORTS = ["sw_create", "sw_destroy", "sw_last_error", "sw_create_batch", "sw_cell_map", "sw_counts",
           "sw_node_coords", "sw_dof_coords", "sw_set_bathymetry", "sw_set_manning", "sw_set_bed_offset",
           "sw_set_state", "sw_get_state", "sw_init_lake_at_rest", "sw_set_time", "sw_apply_operator",
           "sw_apply_operator_noalloc",
           "sw_step_begin", "sw_rk_stage", "sw_step_end", "sw_step", "sw_run", "sw_diagnostics",
           "sw_member_diagnostics", "sw_profile", "sw_kernel_time", "sw_kernel_time_reset", "sw_sync",
           "sw_ens_create", "sw_ens_destroy", "sw_ens_batches", "sw_ens_batch", "sw_ens_member", "sw_ens_run",
           "sw_ens_sync", "sw_vjp_operator", "sw_step_record", "sw_vjp_step", "sw_tracer_step", "sw_locate_points", "sw_boundary_nodes", "sw_set_boundary_state", "sw_set_workgroup", "sw_get_workgroup", "sw_autotune",
           "sw_ens_autotune", "sw_set_bed_grid", "sw_amr_indicator", "sw_remesh", "sw_cells", "sw_amr_plan", "sw_set_tide",
           "sw_ens_step", "sw_step_tracers", "sw_step_tracers_react"]

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.c_void_p


class SwMeshDesc(ctypes.Structure):
    _fields_ = [("nx0", ctypes.c_int32), ("ny0", ctypes.c_int32), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("dx0", ctypes.c_double), ("n_cells", ctypes.c_int32),
                ("level", _c_i32p), ("i", _c_i32p), ("j", _c_i32p), ("bc", ctypes.c_int32 * 4)]


class SwParams(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("rule", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("S", ctypes.c_int32 * 8), ("rk", ctypes.c_int32), ("g", ctypes.c_double),
                ("eps", ctypes.c_double), ("h_lim", ctypes.c_double), ("eps0", ctypes.c_double),
                ("newton_max", ctypes.c_int32), ("cfl", ctypes.c_double), ("cfl_mode", ctypes.c_int32),
                ("tracer", ctypes.c_int32), ("adapt_degree", ctypes.c_int32), ("tide_amp", ctypes.c_double),
                ("tide_period", ctypes.c_double), ("tide_phase", ctypes.c_double), ("tide_c_in", ctypes.c_double),
                ("tracer_diff", ctypes.c_double), ("tracer_strain", ctypes.c_double),
                ("tracer_decay", ctypes.c_double), ("quadrature", ctypes.c_int32)]


class SwAmrParams(ctypes.Structure):
    _fields_ = [("indicator", ctypes.c_int32), ("theta_r", ctypes.c_double), ("theta_c", ctypes.c_double),
                ("n_max", ctypes.c_int32), ("h_min", ctypes.c_double)]


class SwAmrStats(ctypes.Structure):
    _fields_ = [("n_cells_old", ctypes.c_int64), ("n_cells_new", ctypes.c_int64), ("n_refined", ctypes.c_int64),
                ("n_coarsened", ctypes.c_int64), ("eta_max", ctypes.c_double), ("mass_old", ctypes.c_double),
                ("mass_new", ctypes.c_double), ("q_bathy", ctypes.c_double), ("boundary_data_kept", ctypes.c_int32)]


AMR_INDICATOR = {"vorticity": 0, "tracer_grad": 1}


class SwDiag(ctypes.Structure):
    _fields_ = [("total_mass", ctypes.c_double), ("min_target_mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("t", ctypes.c_double), ("n_pos_viol", ctypes.c_int64), ("max_newton_it", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32), ("n_r0_cells", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("step", ctypes.c_int64)]


_LIB = None


def load():
    """Load libswdg.so (raises if it is missing: there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} not found: build it with paper_2505_18743_amd.build.build_library()")
    L = ctypes.CDLL(LIBPATH)
    vp = ctypes.c_void_p
    L.sw_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SwMeshDesc), ctypes.POINTER(SwParams), vp]
    L.sw_create_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(SwMeshDesc),
                                  ctypes.POINTER(SwParams), vp]
    L.sw_cell_map.argtypes = [vp, vp, vp]
    L.sw_member_diagnostics.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(SwDiag)]
    L.sw_ens_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(SwMeshDesc),
                                ctypes.POINTER(SwParams), vp]
    L.sw_ens_destroy.argtypes = [vp]
    L.sw_ens_destroy.restype = None
    L.sw_ens_batches.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.sw_ens_batch.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32)]
    L.sw_ens_member.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.sw_ens_run.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32]
    L.sw_ens_sync.argtypes = [vp]
    L.sw_vjp_operator.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp, vp, vp]
    L.sw_step_record.argtypes = [vp, ctypes.c_double, vp, vp]
    L.sw_tracer_step.argtypes = [vp, vp, vp, ctypes.c_double]
    L.sw_locate_points.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    L.sw_boundary_nodes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp, vp]
    L.sw_set_boundary_state.argtypes = [vp, vp]
    L.sw_set_workgroup.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.sw_get_workgroup.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.sw_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32)]
    L.sw_ens_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p]
    L.sw_vjp_step.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    L.sw_set_bed_grid.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, vp]
    L.sw_amr_indicator.argtypes = [vp, ctypes.c_int32, vp]
    L.sw_remesh.argtypes = [vp, ctypes.POINTER(SwAmrParams), ctypes.POINTER(SwAmrStats)]
    L.sw_cells.argtypes = [vp, vp, vp, vp]
    L.sw_amr_plan.argtypes = [ctypes.POINTER(SwMeshDesc), vp, ctypes.POINTER(SwAmrParams), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32), vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]
    L.sw_destroy.argtypes = [vp]
    L.sw_destroy.restype = None
    L.sw_last_error.restype = ctypes.c_char_p
    L.sw_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int64)]
    L.sw_node_coords.argtypes = [vp, vp]
    L.sw_dof_coords.argtypes = [vp, vp]
    L.sw_set_bathymetry.argtypes = [vp, vp]
    L.sw_set_manning.argtypes = [vp, vp]
    L.sw_set_bed_offset.argtypes = [vp, vp]
    L.sw_set_state.argtypes = [vp, vp, vp, vp, vp]
    L.sw_get_state.argtypes = [vp, vp, vp, vp, vp]
    L.sw_init_lake_at_rest.argtypes = [vp, vp]
    L.sw_set_time.argtypes = [vp, ctypes.c_double]
    L.sw_step_tracers.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_double]
    L.sw_step_tracers_react.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_double]
    L.sw_set_tide.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.sw_ens_step.argtypes = [vp, ctypes.c_int32]
    L.sw_apply_operator.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp]
    L.sw_apply_operator_noalloc.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp]
    L.sw_step_begin.argtypes = [vp, ctypes.c_double]
    L.sw_rk_stage.argtypes = [vp, ctypes.c_int32]
    L.sw_step_end.argtypes = [vp]
    L.sw_step.argtypes = [vp, ctypes.c_double]
    L.sw_run.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.sw_diagnostics.argtypes = [vp, ctypes.POINTER(SwDiag)]
    L.sw_sync.argtypes = [vp]
    L.sw_profile.argtypes = [vp, ctypes.c_int32]
    L.sw_kernel_time.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.sw_kernel_time_reset.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("sw_destroy", "sw_last_error", "sw_ens_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _check(st, what):
    if st != 0:
        msg = load().sw_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed with status {st}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def make_params(pd):
    p = SwParams()
    p.r = int(pd["r"])
    p.rule = RULE[pd.get("rule", "eq")]
    S = list(pd["S"])
    p.n_levels = len(S)
    for k, s in enumerate(S):
        p.S[k] = int(s)
    p.rk = RK[pd.get("rk", "ssp3")]
    p.g = float(pd.get("g", 9.81))
    p.eps = float(pd.get("eps", 0.1))
    p.h_lim = float(pd.get("h_lim", 0.1))
    p.eps0 = float(pd.get("eps0", 1e-8))
    p.newton_max = int(pd.get("newton_max", 20))
    p.cfl = float(pd.get("cfl", 0.2))
    p.cfl_mode = int(pd.get("cfl_mode", 0))
    p.tracer = int(bool(pd.get("tracer", False)))
    p.adapt_degree = int(bool(pd.get("adapt_degree", True)))
    tide = tuple(pd.get("tide", (0.0, 1.0, 0.0, 0.0)))
    p.tide_amp, p.tide_period, p.tide_phase, p.tide_c_in = (float(v) for v in tide)
    p.tracer_diff = float(pd.get("tracer_diff", 0.0))
    p.tracer_strain = float(pd.get("tracer_strain", 0.0))
    p.tracer_decay = float(pd.get("tracer_decay", 0.0))
    p.quadrature = QUADRATURE[pd.get("quadrature", "subgrid")]
    return p


def amr_plan(mesh, eta, indicator="vorticity", theta_r=1e-4, theta_c=5e-5, n_max=2, h_min=0.0):
    """sw_amr_plan: the mesh decision of sw_remesh on the host.  Returns a dict
    with the new leaves (level, i, j), the source kind (type) and cells (src
    [n, 4]) of each, and the refine / merge counts."""
    keep = []
    md = make_mesh(mesh, keep)
    e = np.ascontiguousarray(eta, dtype=np.float64)
    ap = SwAmrParams(AMR_INDICATOR[indicator], float(theta_r), float(theta_c), int(n_max), float(h_min))
    n = ctypes.c_int32(0)
    nr, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    L = load()
    st = L.sw_amr_plan(ctypes.byref(md), e.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ap), 0, ctypes.byref(n),
                       None, None, None, None, None, ctypes.byref(nr), ctypes.byref(nc))
    cap = n.value
    out = {k: np.zeros(cap, dtype=np.int32) for k in ("level", "i", "j", "type")}
    src = np.zeros((cap, 4), dtype=np.int32)
    _check(L.sw_amr_plan(ctypes.byref(md), e.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ap), cap,
                         ctypes.byref(n), *[out[k].ctypes.data_as(ctypes.c_void_p) for k in ("level", "i", "j", "type")],
                         src.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nr), ctypes.byref(nc)), "sw_amr_plan")
    del st
    out.update(src=src, n_refined=nr.value, n_coarsened=nc.value)
    return out


def make_mesh(mesh, keep):
    """sw_mesh_desc of a mesh dict; the index arrays are appended to `keep`."""
    lev = np.ascontiguousarray(mesh["level"], dtype=np.int32)
    ii = np.ascontiguousarray(mesh["i"], dtype=np.int32)
    jj = np.ascontiguousarray(mesh["j"], dtype=np.int32)
    keep += [lev, ii, jj]
    d = SwMeshDesc()
    d.nx0, d.ny0 = int(mesh["nx0"]), int(mesh["ny0"])
    d.x0, d.y0, d.dx0 = float(mesh["x0"]), float(mesh["y0"]), float(mesh["dx0"])
    d.n_cells = len(lev)
    d.level = lev.ctypes.data_as(_c_i32p)
    d.i = ii.ctypes.data_as(_c_i32p)
    d.j = jj.ctypes.data_as(_c_i32p)
    for k, b in enumerate(mesh["bc"]):
        d.bc[k] = BC[b]
    return d


class Solver:
    """One context of the HIP library on one device and stream.

    `mesh` and `params` are one mesh dict and one parameter dict, or lists of
    them (a batched context of independent members, sw_create_batch)."""

    def __init__(self, mesh, params, device="cuda:0", _handle=None):
        L = load()
        self.dev = torch.device(device)
        batched = isinstance(mesh, (list, tuple))
        meshes = list(mesh) if batched else [mesh]
        plist = list(params) if batched else [params]
        self.meshes, self.plist = meshes, plist
        self.params = dict(plist[0])
        self.n_members = len(meshes)
        self._owned = _handle is None
        with torch.cuda.device(self.dev):
            self.stream = torch.cuda.current_stream(self.dev)
            if _handle is None:
                keep = []
                md = (SwMeshDesc * len(meshes))(*[make_mesh(m, keep) for m in meshes])
                pp = (SwParams * len(plist))(*[make_params(q) for q in plist])
                h = ctypes.c_void_p()
                if batched:
                    _check(L.sw_create_batch(ctypes.byref(h), len(meshes), md, pp,
                                             ctypes.c_void_p(self.stream.cuda_stream)), "sw_create_batch")
                else:
                    _check(L.sw_create(ctypes.byref(h), md, pp, ctypes.c_void_p(self.stream.cuda_stream)),
                           "sw_create")
            else:
                h = _handle
        self.h = h
        nc, nv, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.sw_counts(self.h, ctypes.byref(nc), ctypes.byref(nv), ctypes.byref(nd)), "sw_counts")
        self.n_cells, self.n_vol, self.n_dofs = nc.value, nv.value, nd.value
        self.np_ = self.n_dofs // self.n_cells
        self.tracer = bool(self.params.get("tracer", False))
        self._member_index = None

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                load().sw_destroy(self.h)
            self.h = None

    # ---- members of a batched context ----
    def cell_map(self):
        """(member, index in the member's description) of every context cell."""
        mem = np.zeros(self.n_cells, dtype=np.int32)
        loc = np.zeros(self.n_cells, dtype=np.int32)
        _check(load().sw_cell_map(self.h, mem.ctypes.data_as(ctypes.c_void_p), loc.ctypes.data_as(ctypes.c_void_p)),
               "sw_cell_map")
        return mem, loc

    def member_index(self, m):
        """Index arrays (cells, sample nodes, nodal values) of member m in
        context order, listed in the member's own order."""
        if self._member_index is None:
            mem, loc = self.cell_map()
            S = list(self.params["S"])
            lev_ctx = np.empty(self.n_cells, dtype=np.int64)
            for k in range(self.n_members):
                sel = mem == k
                lev_ctx[sel] = np.asarray(self.meshes[k]["level"])[loc[sel]]
            nn = np.asarray(S, dtype=np.int64)[lev_ctx] ** 2
            noff = np.concatenate([[0], np.cumsum(nn)])
            out = []
            for k in range(self.n_members):
                cells = np.nonzero(mem == k)[0]
                cells = cells[np.argsort(loc[cells], kind="stable")]
                cnt = nn[cells]
                start = np.repeat(noff[cells], cnt)
                ofs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                nodes = start + ofs
                dofs = (cells[:, None] * self.np_ + np.arange(self.np_)[None, :]).reshape(-1)
                out.append((cells, nodes, dofs))
            self._member_index = out
        return self._member_index[m]

    def gather_members(self, arrays, kind):
        """Context-order tensor from per-member arrays (kind: 'cells', 'nodes' or 'dofs')."""
        n = {"cells": self.n_cells, "nodes": self.n_vol, "dofs": self.n_dofs}[kind]
        col = {"cells": 0, "nodes": 1, "dofs": 2}[kind]
        full = torch.zeros(n, dtype=torch.float64, device=self.dev)
        for m, a in enumerate(arrays):
            idx = torch.as_tensor(self.member_index(m)[col], device=self.dev)
            full[idx] = self._dev(a, idx.numel())
        return full

    def member_part(self, t, m, kind):
        col = {"cells": 0, "nodes": 1, "dofs": 2}[kind]
        return t[torch.as_tensor(self.member_index(m)[col], device=self.dev)]

    def locate_points(self, xy, member=0):
        """(cell, phi): containing cell and basis values of each point."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        cell = np.zeros(len(xy), dtype=np.int32)
        phi = np.zeros((len(xy), self.np_))
        _check(load().sw_locate_points(self.h, int(member), len(xy), xy.ctypes.data_as(ctypes.c_void_p),
                                       cell.ctypes.data_as(ctypes.c_void_p), phi.ctypes.data_as(ctypes.c_void_p)),
               "sw_locate_points")
        return cell, phi

    def boundary_nodes(self):
        """(xy [n, 2], member [n]) of the face nodes of the state and discharge sides."""
        n = ctypes.c_int64(0)
        _check(load().sw_boundary_nodes(self.h, ctypes.byref(n), None, None), "sw_boundary_nodes")
        xy = np.zeros((n.value, 2))
        mem = np.zeros(n.value, dtype=np.int32)
        if n.value:
            _check(load().sw_boundary_nodes(self.h, ctypes.byref(n), xy.ctypes.data_as(ctypes.c_void_p),
                                            mem.ctypes.data_as(ctypes.c_void_p)), "sw_boundary_nodes")
        return xy, mem

    def set_boundary_state(self, given):
        """Given boundary data: a [4, n] array (zeta, qx, qy, c per boundary
        node) or a function fn(x, y) -> (zeta, qx, qy, c) sampled at the nodes."""
        if callable(given):
            xy, _ = self.boundary_nodes()
            vals = given(xy[:, 0], xy[:, 1])
            given = np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), (len(xy),)) for v in vals])
        n = ctypes.c_int64(0)
        _check(load().sw_boundary_nodes(self.h, ctypes.byref(n), None, None), "sw_boundary_nodes")
        t = self._dev(given, 4 * n.value)
        _check(load().sw_set_boundary_state(self.h, _ptr(t)), "sw_set_boundary_state")
        self._ghost = t        # kept alive until the copy has run

    def member_diagnostics(self, m):
        d = SwDiag()
        _check(load().sw_member_diagnostics(self.h, int(m), ctypes.byref(d)), "sw_member_diagnostics")
        return {k: getattr(d, k) for k, _ in SwDiag._fields_}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers ----
    def _dev(self, a, n=None):
        t = torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a, dtype=torch.float64)
        t = t.to(self.dev).contiguous().reshape(-1)
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def zeros(self):
        return torch.zeros(self.n_dofs, dtype=torch.float64, device=self.dev)

    # ---- setup ----
    def node_coords(self):
        xy = np.zeros((self.n_vol, 2))
        _check(load().sw_node_coords(self.h, xy.ctypes.data_as(ctypes.c_void_p)), "sw_node_coords")
        return xy

    def dof_coords(self):
        xy = np.zeros((self.n_dofs, 2))
        _check(load().sw_dof_coords(self.h, xy.ctypes.data_as(ctypes.c_void_p)), "sw_dof_coords")
        return xy

    def set_bathymetry(self, b):
        t = self._dev(b, self.n_vol)
        _check(load().sw_set_bathymetry(self.h, _ptr(t)), "sw_set_bathymetry")
        self._keep = t

    def set_manning(self, n):
        t = self._dev(n, self.n_cells)
        _check(load().sw_set_manning(self.h, _ptr(t)), "sw_set_manning")
        self._keep_n = t

    def set_bed_offset(self, db):
        t = self._dev(db, self.n_cells)
        _check(load().sw_set_bed_offset(self.h, _ptr(t)), "sw_set_bed_offset")
        self._keep_db = t

    def set_state(self, eta, qx, qy, c=None):
        ts = [self._dev(a, self.n_dofs) for a in (eta, qx, qy)]
        tc = self._dev(c, self.n_dofs) if c is not None else None
        _check(load().sw_set_state(self.h, *[_ptr(t) for t in ts], _ptr(tc)), "sw_set_state")
        self._keep_s = (ts, tc)

    def get_state(self):
        out = [self.zeros() for _ in range(4)]
        _check(load().sw_get_state(self.h, *[_ptr(t) for t in out]), "sw_get_state")
        return out

    def init_lake_at_rest(self, eta):
        t = self._dev(eta, self.n_dofs)
        _check(load().sw_init_lake_at_rest(self.h, _ptr(t)), "sw_init_lake_at_rest")
        self._keep_l = t

    def set_time(self, t):
        _check(load().sw_set_time(self.h, float(t)), "sw_set_time")

    def set_tide(self, amplitude, period, phase=0.0, c_inflow=0.0):
        """sw_set_tide: the elevation boundary's tide of every member."""
        _check(load().sw_set_tide(self.h, float(amplitude), float(period), float(phase), float(c_inflow)),
               "sw_set_tide")

    # ---- operator and stepping ----
    def apply_operator(self, eta, qx, qy, c=None, t=0.0):
        ins = [self._dev(a, self.n_dofs) for a in (eta, qx, qy)]
        tc = self._dev(c, self.n_dofs) if c is not None else self.zeros()
        outs = [self.zeros() for _ in range(4)]
        dtb = torch.zeros(1, dtype=torch.float64, device=self.dev)
        _check(load().sw_apply_operator(self.h, *[_ptr(x) for x in ins], _ptr(tc), float(t),
                                        *[_ptr(x) for x in outs], _ptr(dtb)), "sw_apply_operator")
        return outs[0], outs[1], outs[2], outs[3], dtb

    def apply_operator_noalloc(self, eta, qx, qy, c, t, out):
        """sw_apply_operator_noalloc: the residuals of sw_apply_operator with the
        call's device scratch in the library's fixed array (no allocation by
        the library).  eta, qx, qy, c: device float64 [n_dofs] (c may be None
        without a tracer); out = (F, Gx, Gy, R, dtb): caller-owned device
        float64 tensors ([n_dofs] each, R may be None without a tracer; dtb [1]
        or None), written in place."""
        ins = [self._dev(a, self.n_dofs) for a in (eta, qx, qy)]
        tc = self._dev(c, self.n_dofs) if c is not None else None
        for o in out:
            if o is not None and (not self._on_dev(o) or o.dtype != torch.float64 or not o.is_contiguous()):
                raise ValueError("outputs must be contiguous float64 tensors on the solver's device")
        for o in out[:4]:
            if o is not None and o.numel() != self.n_dofs:
                raise ValueError("residual outputs must hold n_dofs values")
        _check(load().sw_apply_operator_noalloc(self.h, *[_ptr(x) for x in ins], _ptr(tc), float(t),
                                                *[_ptr(x) for x in out]), "sw_apply_operator_noalloc")

    def step_begin(self, dt=0.0):
        _check(load().sw_step_begin(self.h, float(dt)), "sw_step_begin")

    def rk_stage(self, l):
        _check(load().sw_rk_stage(self.h, int(l)), "sw_rk_stage")

    def step_end(self):
        _check(load().sw_step_end(self.h), "sw_step_end")

    def step(self, dt=0.0):
        _check(load().sw_step(self.h, float(dt)), "sw_step")

    def run(self, n, dt=0.0):
        _check(load().sw_run(self.h, int(n), float(dt)), "sw_run")

    def sync(self):
        _check(load().sw_sync(self.h), "sw_sync")

    def step_tracers(self, tracers, dt):
        """sw_step_tracers: one fixed-dt step of this (flow) context and of the
        given tracer Solvers over its recorded flow."""
        arr = (ctypes.c_void_p * max(len(tracers), 1))(*[t.h for t in tracers])
        _check(load().sw_step_tracers(self.h, len(tracers), arr, float(dt)), "sw_step_tracers")

    def step_tracers_react(self, tracers, react, dt):
        """sw_step_tracers_react: step_tracers with the linear reactions
        phi_k = sum_j react[k][j] c_j between the given tracer Solvers (react:
        an n x n matrix, 1/s)."""
        n = len(tracers)
        B = np.ascontiguousarray(np.asarray(react, dtype=np.float64).reshape(n, n))
        arr = (ctypes.c_void_p * max(n, 1))(*[t.h for t in tracers])
        _check(load().sw_step_tracers_react(self.h, n, arr, B.ctypes.data_as(ctypes.c_void_p), float(dt)),
               "sw_step_tracers_react")

    # ---- dynamic h-adaptivity ----
    def set_bed_grid(self, grid):
        """Bathymetry raster: grid = dict(x0, y0, dx, dy, b [ny, nx]) of bed
        elevations; sampled at every node now and after every remesh."""
        b = np.asarray(grid["b"], dtype=np.float64)
        ny, nx = b.shape
        t = self._dev(b, nx * ny)
        _check(load().sw_set_bed_grid(self.h, int(nx), int(ny), float(grid["x0"]), float(grid["y0"]),
                                      float(grid["dx"]), float(grid["dy"]), _ptr(t)), "sw_set_bed_grid")
        self._keep_g = t

    def amr_indicator(self, kind="vorticity"):
        eta = torch.zeros(self.n_cells, dtype=torch.float64, device=self.dev)
        _check(load().sw_amr_indicator(self.h, AMR_INDICATOR[kind], _ptr(eta)), "sw_amr_indicator")
        return eta

    def cells(self):
        """(level, i, j) of every cell."""
        out = [np.zeros(self.n_cells, dtype=np.int32) for _ in range(3)]
        _check(load().sw_cells(self.h, *[o.ctypes.data_as(ctypes.c_void_p) for o in out]), "sw_cells")
        return out

    def remesh(self, indicator="vorticity", theta_r=1e-4, theta_c=5e-5, n_max=2, h_min=0.0):
        """sw_remesh; returns its statistics.  Sizes and the mesh description
        follow the new mesh."""
        ap = SwAmrParams(AMR_INDICATOR[indicator], float(theta_r), float(theta_c), int(n_max), float(h_min))
        st = SwAmrStats()
        _check(load().sw_remesh(self.h, ctypes.byref(ap), ctypes.byref(st)), "sw_remesh")
        nc, nv, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().sw_counts(self.h, ctypes.byref(nc), ctypes.byref(nv), ctypes.byref(nd)), "sw_counts")
        self.n_cells, self.n_vol, self.n_dofs = nc.value, nv.value, nd.value
        lev, ii, jj = self.cells()
        self.meshes[0] = dict(self.meshes[0], level=lev, i=ii, j=jj)
        self._member_index = None
        return {k: getattr(st, k) for k, _ in SwAmrStats._fields_}

    # ---- adjoint ----
    def vjp_operator(self, eta, qx, qy, Fb, Gxb, Gyb, t=0.0):
        """(eta_b, qx_b, qy_b, n_bar, db_bar): transpose of the residual Jacobian."""
        ins = [self._dev(a, self.n_dofs) for a in (eta, qx, qy, Fb, Gxb, Gyb)]
        outs = [self.zeros() for _ in range(3)]
        pb = [torch.zeros(self.n_cells, dtype=torch.float64, device=self.dev) for _ in range(2)]
        _check(load().sw_vjp_operator(self.h, *[_ptr(x) for x in ins[:3]], float(t), *[_ptr(x) for x in ins[3:]],
                                      *[_ptr(x) for x in outs], *[_ptr(x) for x in pb]), "sw_vjp_operator")
        return outs[0], outs[1], outs[2], pb[0], pb[1]

    def n_stages(self):
        return {"fe": 1, "ssp3": 3, "rk32": 3, "rk44": 4, "imex": 3}[self.params.get("rk", "ssp3")]

    def _on_dev(self, x):
        """x is a tensor on the solver's GPU."""
        return (torch.is_tensor(x) and x.device.type == "cuda"
                and (self.dev.index is None or x.device.index == self.dev.index))

    def _flow_buf(self, x, n, what):
        if (not torch.is_tensor(x) or x.numel() != n * 3 * self.n_dofs or not x.is_contiguous()
                or x.dtype != torch.float64 or x.device.type != "cuda"):
            raise ValueError(f"{what} must be a contiguous float64 device tensor of {n} x 3 x n_dofs")

    def step_record(self, dt, stages, end=None):
        """One fixed-dt step storing its stage states into `stages` [s, 3, n_dofs]
        and, if given, the final combination's flow into `end` [3, n_dofs]."""
        self._flow_buf(stages, self.n_stages(), "stages")
        if end is not None:
            self._flow_buf(end, 1, "end")
        _check(load().sw_step_record(self.h, float(dt), _ptr(stages), _ptr(end)),
               "sw_step_record")

    def tracer_step(self, stages, end, dt):
        """Advance the tracer by one recorded step (flow from `stages`, `end`)."""
        self._flow_buf(stages, self.n_stages(), "stages")
        self._flow_buf(end, 1, "end")
        _check(load().sw_tracer_step(self.h, _ptr(stages), _ptr(end), float(dt)), "sw_tracer_step")

    def vjp_step(self, stages, t, dt, state_bar, n_bar, db_bar):
        """Adjoint of one recorded step: state_bar [3, n_dofs] updated in place
        (adjoint of u^(n+1) -> of u^n); n_bar, db_bar [n_cells] accumulated.
        Every array is a device tensor on the solver's device (the kernels
        read and write them directly)."""
        self._flow_buf(stages, self.n_stages(), "stages")
        if not self._on_dev(stages):
            raise ValueError("stages must live on the solver's device")
        for x, n in ((state_bar, 3 * self.n_dofs), (n_bar, self.n_cells), (db_bar, self.n_cells)):
            if (not torch.is_tensor(x) or x.numel() != n or not x.is_contiguous() or x.dtype != torch.float64
                    or not self._on_dev(x)):
                raise ValueError("adjoint arrays must be contiguous float64 tensors of the right size "
                                 "on the solver's device")
        _check(load().sw_vjp_step(self.h, _ptr(stages), float(t), float(dt), _ptr(state_bar), _ptr(n_bar),
                                  _ptr(db_bar)), "sw_vjp_step")

    def set_workgroup(self, value, level=-1, kernel=0):
        """Launch shape: kernel 0 = fast element kernel, value = wavefronts
        per workgroup (1, 2, 4); kernel 1 = face kernel, value = lanes per face
        (2, 4, 8); kernel 2 = fast-kernel cell order over the XCDs (0 round
        robin, 1 contiguous ranges, -1 by the mesh)."""
        _check(load().sw_set_workgroup(self.h, int(level), int(kernel), int(value)), "sw_set_workgroup")

    def get_workgroup(self, level=0, kernel=0):
        v = ctypes.c_int32()
        _check(load().sw_get_workgroup(self.h, int(level), int(kernel), ctypes.byref(v)), "sw_get_workgroup")
        return v.value

    def autotune(self, steps=8, dt=0.0):
        """Time every launch shape on the current state, keep the fastest."""
        w, q = ctypes.c_int32(), ctypes.c_int32()
        _check(load().sw_autotune(self.h, int(steps), float(dt), ctypes.byref(w), ctypes.byref(q)), "sw_autotune")
        return dict(elem_waves_per_workgroup=w.value, face_lanes=q.value, elem_order=self.get_workgroup(0, 2))

    def profile(self, on=True, kinds=None):
        """Kernel timing on/off; kinds: names of KERNELS to time (default all)."""
        v = int(bool(on))
        if on and kinds:
            mask = sum(1 << self.KERNELS.index(k) for k in kinds)
            v = 1 | (mask << 1)
        _check(load().sw_profile(self.h, v), "sw_profile")

    KERNELS = ("element_start", "element_stage", "element_final", "face", "element_general", "element_tracer",
               "element_tracer_final", "reactions")

    def kernel_times(self):
        """{kernel class: (total ms, launches)} accumulated while profiling."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(load().sw_kernel_time(self.h, k, ctypes.byref(ms), ctypes.byref(n)), "sw_kernel_time")
            out[name] = (ms.value, n.value)
        return out

    def kernel_time_reset(self):
        _check(load().sw_kernel_time_reset(self.h), "sw_kernel_time_reset")

    def diagnostics(self):
        d = SwDiag()
        _check(load().sw_diagnostics(self.h, ctypes.byref(d)), "sw_diagnostics")
        return {k: getattr(d, k) for k, _ in SwDiag._fields_}


class Ensemble:
    """Independent members grouped into batched contexts (sw_ens_create);
    member arrays go in and out in each member's own layout."""

    def __init__(self, meshes, params, device="cuda:0"):
        L = load()
        self.dev = torch.device(device)
        self.meshes, self.plist = list(meshes), list(params)
        self.n_members = len(self.meshes)
        with torch.cuda.device(self.dev):
            self.stream = torch.cuda.current_stream(self.dev)
            keep = []
            md = (SwMeshDesc * self.n_members)(*[make_mesh(m, keep) for m in self.meshes])
            pp = (SwParams * self.n_members)(*[make_params(q) for q in self.plist])
            h = ctypes.c_void_p()
            _check(L.sw_ens_create(ctypes.byref(h), self.n_members, md, pp,
                                   ctypes.c_void_p(self.stream.cuda_stream)), "sw_ens_create")
        self.h = h
        nb = ctypes.c_int32()
        _check(L.sw_ens_batches(self.h, ctypes.byref(nb)), "sw_ens_batches")
        self.where = []
        for m in range(self.n_members):
            b, i = ctypes.c_int32(), ctypes.c_int32()
            _check(L.sw_ens_member(self.h, m, ctypes.byref(b), ctypes.byref(i)), "sw_ens_member")
            self.where.append((b.value, i.value))
        self.batches = []
        for b in range(nb.value):
            c, n = ctypes.c_void_p(), ctypes.c_int32()
            _check(L.sw_ens_batch(self.h, b, ctypes.byref(c), ctypes.byref(n)), "sw_ens_batch")
            mem = [m for m in range(self.n_members) if self.where[m][0] == b]
            self.batches.append(Solver([self.meshes[m] for m in mem], [self.plist[m] for m in mem], device,
                                       _handle=c))

    def close(self):
        if getattr(self, "h", None):
            for s in self.batches:
                s.h = None
            load().sw_ens_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _per_batch(self, arrays):
        out = [[] for _ in self.batches]
        for m, a in enumerate(arrays):
            out[self.where[m][0]].append(a)
        return out

    def member_coords(self, m, kind="nodes"):
        b, i = self.where[m]
        s = self.batches[b]
        xy = s.node_coords() if kind == "nodes" else s.dof_coords()
        col = 1 if kind == "nodes" else 2
        return xy[s.member_index(i)[col]]

    def set_bathymetry(self, arrays):
        for s, arr in zip(self.batches, self._per_batch(arrays)):
            s.set_bathymetry(s.gather_members(arr, "nodes"))

    def set_manning(self, arrays):
        for s, arr in zip(self.batches, self._per_batch(arrays)):
            s.set_manning(s.gather_members(arr, "cells"))

    def init_lake_at_rest(self, arrays):
        for s, arr in zip(self.batches, self._per_batch(arrays)):
            s.init_lake_at_rest(s.gather_members(arr, "dofs"))

    def set_time(self, t):
        for s in self.batches:
            s.set_time(t)

    def get_state(self, m):
        b, i = self.where[m]
        s = self.batches[b]
        return [s.member_part(x, i, "dofs") for x in s.get_state()]

    def locate_points(self, xy, member=0):
        """(cell, phi): containing cell and basis values of each point."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        cell = np.zeros(len(xy), dtype=np.int32)
        phi = np.zeros((len(xy), self.np_))
        _check(load().sw_locate_points(self.h, int(member), len(xy), xy.ctypes.data_as(ctypes.c_void_p),
                                       cell.ctypes.data_as(ctypes.c_void_p), phi.ctypes.data_as(ctypes.c_void_p)),
               "sw_locate_points")
        return cell, phi

    def member_diagnostics(self, m):
        b, i = self.where[m]
        return self.batches[b].member_diagnostics(i)

    def run(self, n, dt=0.0, graph=True):
        _check(load().sw_ens_run(self.h, int(n), float(dt), int(bool(graph))), "sw_ens_run")

    def step(self, graph=True):
        """sw_ens_step: one step of every member with its CFL time step."""
        _check(load().sw_ens_step(self.h, int(bool(graph))), "sw_ens_step")

    def autotune(self, steps=8, cache=None):
        """Launch-shape autotuner of every batch; returns the chosen shapes."""
        _check(load().sw_ens_autotune(self.h, int(steps), (cache or "").encode()), "sw_ens_autotune")
        return [dict(r=s.params["r"], elem_waves_per_workgroup=s.get_workgroup(0, 0),
                     face_lanes=s.get_workgroup(0, 1)) for s in self.batches]

    def sync(self):
        _check(load().sw_ens_sync(self.h), "sw_ens_sync")
