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


def ensemble_inputs(ens, members):
    """Context-order inputs of every batch of an Ensemble built from workload
    member dicts: bed at the sample nodes (sampled on the device), Manning per
    cell, Def. 3.1 initial state from eta0.  Returns [(bed, manning, eta)]."""
    import torch
    out = []
    for b, s in enumerate(ens.batches):
        mem = [m for m in range(len(members)) if ens.where[m][0] == b]
        xy = torch.as_tensor(s.node_coords(), device=s.dev)
        dxy = s.dof_coords()
        bed = torch.zeros(s.n_vol, dtype=torch.float64, device=s.dev)
        man = torch.zeros(s.n_cells, dtype=torch.float64, device=s.dev)
        eta = torch.zeros(s.n_dofs, dtype=torch.float64, device=s.dev)
        for i, m in enumerate(mem):
            cells, nodes, dofs = s.member_index(i)
            w = members[m]
            nt = torch.as_tensor(nodes, device=s.dev)
            bed[nt] = w["bed"](xy[nt, 0], xy[nt, 1])
            man[torch.as_tensor(cells, device=s.dev)] = torch.as_tensor(np.asarray(w["manning"], dtype=np.float64),
                                                                        device=s.dev)
            eta[torch.as_tensor(dofs, device=s.dev)] = torch.as_tensor(
                np.asarray(w["eta0"](dxy[dofs, 0], dxy[dofs, 1]), dtype=np.float64), device=s.dev)
        out.append((bed, man, eta))
    return out


def setup_ensemble(members, device="cuda:0"):
    """Ensemble of workload member dicts with their inputs in place, time 0."""
    from paper_2505_18743_amd import Ensemble
    ens = Ensemble([w["mesh"] for w in members], [w["params"] for w in members], device)
    inputs = ensemble_inputs(ens, members)
    for s, (bed, man, eta) in zip(ens.batches, inputs):
        s.set_bathymetry(bed)
        s.set_manning(man)
        s.init_lake_at_rest(eta)
        s.set_time(0.0)
    return ens, inputs


def member_solver(ens, inputs, members, m, device="cuda:0"):
    """A one-member context of member m with exactly the ensemble's inputs."""
    from paper_2505_18743_amd import Solver
    b, i = ens.where[m]
    s = ens.batches[b]
    cells, nodes, dofs = s.member_index(i)
    bed, man, eta = inputs[b]
    w = members[m]
    one = Solver(w["mesh"], w["params"], device)
    one.set_bathymetry(bed[nodes])
    one.set_manning(man[cells])
    one.init_lake_at_rest(eta[dofs])
    one.set_time(0.0)
    return one
