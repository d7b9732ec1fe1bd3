"""GPU: batched contexts and ensembles.

A member of a batched context runs the same kernels, cell by cell and face by
face, as a context of its own; only the grouping of cells into launches and
the order of the (exact) minimum reductions differ.  So every member of a
batch must equal its one-by-one run bit for bit, with and without the
captured hipGraph, and the one-by-one runs are tied to the oracle by the
parity tests (and, for two small members, again here).
"""
import numpy as np
import pytest
import torch

from helpers import build_oracle, member_solver, setup_ensemble
from workloads import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(g, r):
    g = np.asarray(g).ravel()
    r = np.asarray(r).ravel()
    scale = np.abs(r).max()
    return np.abs(g - r).max() / (scale if scale > 0 else 1.0)


def same(a, b):
    return torch.equal(a, b)


def small_members(n=6, nmin=3, nmax=9):
    return workload("ensemble_64", members=n, nmin=nmin, nmax=nmax)


def test_ensemble_groups_by_degree():
    say("case: ensemble grouping, 6 small members")
    mem = small_members()
    ens, _ = setup_ensemble(mem)
    rs = sorted({w["params"]["r"] for w in mem})
    assert len(ens.batches) == len(rs)
    for m, w in enumerate(mem):
        b, i = ens.where[m]
        assert ens.batches[b].params["r"] == w["params"]["r"]
        cells, nodes, dofs = ens.batches[b].member_index(i)
        N = w["mesh"]["nx0"]
        assert len(cells) == N * N and len(nodes) == N * N * 256
        # member coordinates are those of a one-member context
    ens.close()


@pytest.mark.parametrize("graph,rk", [(True, None), (False, None), (True, "imex")])
def test_ensemble_equals_one_by_one(graph, rk):
    say(f"case: ensemble vs one-by-one, graph={graph}, rk={rk or 'members own'}, 6 small members, 8 steps")
    mem = small_members()
    if rk is not None:
        for w in mem:
            w["params"] = dict(w["params"], rk=rk)
    ens, inputs = setup_ensemble(mem)
    ens.run(3, graph=graph)
    ens.run(5, graph=graph)
    ens.sync()
    for m, w in enumerate(mem):
        one = member_solver(ens, inputs, mem, m)
        one.run(8)
        one.sync()
        a = ens.get_state(m)
        b = one.get_state()
        for f in range(3):
            assert same(a[f], b[f]), (m, f, float((a[f] - b[f]).abs().max()))
        da, db = ens.member_diagnostics(m), one.diagnostics()
        assert da["t"] == db["t"] and da["dt"] == db["dt"], (m, da, db)
        assert da["total_mass"] == pytest.approx(db["total_mass"], rel=1e-13)
        assert da["max_newton_it"] == db["max_newton_it"]
        one.close()
    ens.close()


def test_ensemble_members_fixed_dt_and_restart():
    say("case: ensemble fixed dt, graph replay after re-initialisation")
    mem = small_members(4, 4, 7)
    ens, inputs = setup_ensemble(mem)
    ens.run(4, dt=0.5, graph=True)
    # re-initialise every batch: the next run takes one eager step, then replays
    for s, (bed, man, eta) in zip(ens.batches, inputs):
        s.init_lake_at_rest(eta)
        s.set_time(0.0)
    ens.run(6, dt=0.5, graph=True)
    ens.sync()
    for m in range(len(mem)):
        one = member_solver(ens, inputs, mem, m)
        one.run(6, 0.5)
        one.sync()
        a, b = ens.get_state(m), one.get_state()
        for f in range(3):
            assert same(a[f], b[f]), (m, f)
        assert ens.member_diagnostics(m)["t"] == pytest.approx(3.0, rel=1e-15)
        one.close()
    ens.close()


def test_ensemble_member_matches_oracle():
    say("case: two ensemble members vs the oracle, 5 steps")
    mem = small_members(6, 3, 6)
    ens, _ = setup_ensemble(mem)
    ens.run(5, graph=True)
    ens.sync()
    for m in range(2):
        o, _ = build_oracle(mem[m])
        for _ in range(5):
            o.step()
        st = o.get_state()
        g = ens.get_state(m)
        K = o.m.K
        for f in range(3):
            e = rel(g[f].cpu().numpy(), st[f])
            say(f"  member {m} r={mem[m]['params']['r']} field {f} rel err {e:.3e}")
            assert e < 1e-10, (m, f, e)
        d = ens.member_diagnostics(m)
        assert d["t"] == pytest.approx(float(o.t), rel=1e-12)
    ens.close()


def hanging_members():
    """Three quadtree members (tracer, RK32, elevation boundary) of one batch:
    different coarse cell sizes, tides and CFL numbers."""
    from workloads import quadtree_desc
    out = []
    for k, (dx0, amp, cfl) in enumerate(((400.0, 0.3, 0.5), (250.0, 0.5, 0.4), (333.0, 0.2, 0.45))):
        def refine(L, cand, k=k):
            return [c for c in cand if (c[1] * (5 + k) + c[2] * 3) % 4 == 0]
        d = quadtree_desc(5 + k, 4 + k, 10.0 * k, -5.0 * k, dx0, refine, 1, bc=("elev", "wall", "open", "wall"))
        params = dict(r=2, S=(16, 8), rule="eq", rk="rk32", g=9.81, eps=0.05, h_lim=0.05, eps0=1e-8,
                      newton_max=20, cfl=cfl, cfl_mode=1, tracer=True, tide=(amp, 3000.0, 0.2 * k, 0.25))
        Lx = d["nx0"] * dx0

        def bed(x, y, Lx=Lx, k=k):
            return -3.0 + 4.5 * x / Lx + 0.6 * np.sin(y / (150.0 + 10 * k)) * np.cos(x / 90.0)

        def eta0(x, y, k=k):
            return 0.4 * np.exp(-((x - 700) ** 2 + (y - 600 - 50 * k) ** 2) / 300.0 ** 2)

        out.append(dict(mesh=d, params=params, bed=bed, eta0=eta0, manning=np.full(len(d["level"]), 0.03 + 0.002 * k)))
    return out


def test_batched_context_hanging_tracer():
    say("case: batched context of 3 quadtree members with tracer, RK32, 6 steps + operator")
    from paper_2505_18743_amd import Solver
    mem = hanging_members()
    s = Solver([w["mesh"] for w in mem], [w["params"] for w in mem], "cuda:0")
    xy = s.node_coords()
    dxy = s.dof_coords()
    beds, mans, etas, trs = [], [], [], []
    for i, w in enumerate(mem):
        cells, nodes, dofs = s.member_index(i)
        beds.append(w["bed"](xy[nodes, 0], xy[nodes, 1]))
        mans.append(w["manning"])
        etas.append(w["eta0"](dxy[dofs, 0], dxy[dofs, 1]))
        trs.append(np.exp(-((dxy[dofs, 0] - 900) ** 2 + (dxy[dofs, 1] - 700) ** 2) / 400.0 ** 2))
    s.set_bathymetry(s.gather_members(beds, "nodes"))
    s.set_manning(s.gather_members(mans, "cells"))
    s.init_lake_at_rest(s.gather_members(etas, "dofs"))
    st = s.get_state()
    s.set_state(st[0], st[1], st[2], s.gather_members(trs, "dofs"))
    s.set_time(0.0)
    st0 = s.get_state()
    ops = s.apply_operator(st0[0], st0[1], st0[2], st0[3], 100.0)
    s.run(6)
    s.sync()
    for i, w in enumerate(mem):
        one = Solver(w["mesh"], w["params"], "cuda:0")
        one.set_bathymetry(beds[i])
        one.set_manning(mans[i])
        one.init_lake_at_rest(etas[i])
        o = one.get_state()
        one.set_state(o[0], o[1], o[2], trs[i])
        one.set_time(0.0)
        o0 = one.get_state()
        for f in range(4):
            assert same(s.member_part(st0[f], i, "dofs"), o0[f]), (i, f)
        op1 = one.apply_operator(o0[0], o0[1], o0[2], o0[3], 100.0)
        for f in range(4):
            assert same(s.member_part(ops[f], i, "dofs"), op1[f]), ("operator", i, f)
        one.run(6)
        one.sync()
        a, b = s.get_state(), one.get_state()
        for f in range(4):
            assert same(s.member_part(a[f], i, "dofs"), b[f]), ("step", i, f)
        da, db = s.member_diagnostics(i), one.diagnostics()
        assert da["t"] == db["t"] and da["dt"] == db["dt"]
        one.close()
    s.close()


@pytest.mark.slow
def test_full_ensemble_64_sampled_members():
    say("case: full ensemble_64 (64 members), 3 graph steps, 4 sampled members vs one-by-one")
    mem = workload("ensemble_64")
    ens, inputs = setup_ensemble(mem)
    ens.run(3, graph=True)
    ens.sync()
    sizes = [w["mesh"]["nx0"] for w in mem]
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 17, 42})
    for m in pick:
        one = member_solver(ens, inputs, mem, m)
        one.run(3)
        one.sync()
        a, b = ens.get_state(m), one.get_state()
        for f in range(3):
            assert same(a[f], b[f]), (m, f)
        d = ens.member_diagnostics(m)
        assert not d["nonfinite"] and d["t"] == one.diagnostics()["t"]
        say(f"  member {m} N={sizes[m]} r={mem[m]['params']['r']} equal, t={d['t']:.3f}")
        one.close()
    ens.close()


def test_ensemble_autotune_and_cache(tmp_path):
    say("case: ensemble autotune with a cache file, 6 small members")
    mem = small_members()
    ens, inputs = setup_ensemble(mem)
    cache = str(tmp_path / "tune.txt")
    chosen = ens.autotune(steps=2, cache=cache)
    say(f"  chosen {chosen}")
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == len(ens.batches)
    # a second ensemble picks the shapes up from the cache without timing
    ens2, _ = setup_ensemble(mem)
    again = ens2.autotune(steps=2, cache=cache)
    assert again == chosen
    # tuned ensemble vs one-by-one runs (rounding only: face-sum order)
    ens.run(6, graph=True)
    ens.sync()
    for m, w in enumerate(mem):
        one = member_solver(ens, inputs, mem, m)
        one.run(6)
        one.sync()
        a, b = ens.get_state(m), one.get_state()
        for f in range(3):
            d = float((a[f] - b[f]).abs().max()) / max(float(b[f].abs().max()), 1e-300)
            assert d < 1e-10, (m, f, d)
        one.close()
    ens.close()
    ens2.close()


def test_ensemble_step_is_one_run_step():
    say("case: sw_ens_step equals sw_ens_run with one step, 4 small members")
    mem = small_members(4, 3, 6)
    out = []
    for use_step in (False, True):
        ens, _ = setup_ensemble(mem)
        for _ in range(3):
            if use_step:
                ens.step(graph=True)
            else:
                ens.run(1, graph=True)
        ens.sync()
        out.append([ens.get_state(m) for m in range(len(mem))])
        ens.close()
    for a, b in zip(*out):
        for f in range(3):
            assert same(a[f], b[f])
