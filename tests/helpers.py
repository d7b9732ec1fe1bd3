"""Shared test helpers: build the oracle from a workload description."""
from __future__ import annotations

import numpy as np

from oracle import Mesh, Oracle, Params


def mesh_from_desc(d):
    return Mesh(d["nx0"], d["ny0"], d["x0"], d["y0"], d["dx0"], d["level"], d["i"], d["j"], d["bc"])


def params_from_dict(pd, **over):
    q = dict(pd)
    q.update(over)
    q["S"] = tuple(q["S"])
    q["tide"] = tuple(q["tide"])
    return Params(**q)


def build_oracle(wl, **over):
    """Oracle on a workload: bathymetry sampled at the oracle's node coordinates,
    nodal initial state at the basis support points, Def. 3.1 dry rule."""
    mesh = mesh_from_desc(wl["mesh"])
    p = params_from_dict(wl["params"], **over)
    o = Oracle(mesh, p)
    xy = o.node_coords()
    b = wl["bed"](xy[:, 0], xy[:, 1])
    o.set_bathymetry(b)
    o.set_manning(wl["manning"])
    dxy = o.dof_coords()
    eta = wl["eta0"](dxy[..., 0], dxy[..., 1])
    c0 = wl.get("tracer0")
    cvals = c0(dxy[..., 0], dxy[..., 1]) if c0 is not None else np.zeros_like(eta)
    o.set_state(eta, np.zeros_like(eta), np.zeros_like(eta), cvals)
    if wl.get("lake_at_rest", False):
        st = o.get_state()
        o.init_lake_at_rest(eta)
        o.state[3] = o.state[3].new_tensor(st[3])
    return o, b
