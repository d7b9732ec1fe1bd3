"""The library's remesh decision (sw_amr_plan, host code only, no device)
against the oracle's plan (Sec. 3.3 criteria with the 2:1 balance across
faces): identical new leaves in the same order, identical sources of every
new cell and identical refine / merge counts, on random quadtrees with
random indicators, walls and periodic sides, with and without H_min."""
import numpy as np
import pytest

from oracle import Mesh
from oracle.amr import plan


def lib_plan(d, eta, tr, tc, nmax, hmin):
    from paper_2505_18743_amd.binding import amr_plan
    return amr_plan(d, eta, "vorticity", tr, tc, nmax, hmin)


def compare(d, eta, tr, tc, nmax, hmin=0.0):
    m = Mesh(d["nx0"], d["ny0"], d["x0"], d["y0"], d["dx0"], d["level"], d["i"], d["j"], d["bc"])
    nm, rel, nref, ncoa, _ = plan(m, eta, tr, tc, nmax, hmin)
    got = lib_plan(d, eta, tr, tc, nmax, hmin)
    assert np.array_equal(got["level"], nm.level)
    assert np.array_equal(got["i"], nm.ii) and np.array_equal(got["j"], nm.jj)
    assert got["n_refined"] == nref and got["n_coarsened"] == ncoa
    for n, r_ in enumerate(rel):
        t = {"copy": 0, "child": 1, "parent": 2}[r_[0]]
        assert got["type"][n] == t, n
        if t == 0:
            assert got["src"][n, 0] == r_[1]
        elif t == 1:
            assert got["src"][n, 0] == r_[1] and got["src"][n, 1] == 2 * r_[3] + r_[2]
        else:
            assert list(got["src"][n]) == list(r_[1])
    return nref, ncoa


@pytest.mark.parametrize("bc", [("wall",) * 4, ("periodic", "periodic", "wall", "open"),
                                ("periodic", "periodic", "periodic", "periodic")])
def test_plan_matches_the_oracle(bc):
    rng = np.random.default_rng(len(bc[0]) + len(bc[2]))
    total_ref = total_coa = 0
    for trial in range(10):
        # a balanced start: a uniform grid refined twice by the oracle's plan
        m = Mesh.uniform(6, 4, 0.0, 0.0, 10.0, bc=bc)
        for _ in range(int(rng.integers(1, 3))):
            m, _, _, _, _ = plan(m, rng.uniform(size=m.K), 0.6, 0.0, 4)
        d = dict(nx0=m.nx0, ny0=m.ny0, x0=m.x0, y0=m.y0, dx0=m.dx0, level=m.level.astype(np.int32),
                 i=m.ii.astype(np.int32), j=m.jj.astype(np.int32), bc=bc)
        K = m.K
        # smooth bumps plus noise: flagged regions are clustered, as in a real run
        xc = (m.ii + 0.5) / 2.0 ** m.level
        yc = (m.jj + 0.5) / 2.0 ** m.level
        eta = np.exp(-((xc - rng.uniform(0, 6)) ** 2 + (yc - rng.uniform(0, 4)) ** 2)) + 0.05 * rng.uniform(size=K)
        nref, ncoa = compare(d, eta, 0.5, 0.2, 4, hmin=2.0 if trial % 3 == 0 else 0.0)
        total_ref += nref
        total_coa += ncoa
    assert total_ref > 0 and total_coa > 0


def test_plan_on_a_uniform_grid_is_in_row_order():
    from workloads.gen import uniform_mesh_desc
    d = uniform_mesh_desc(8, 5, 0.0, 0.0, 1.0)
    eta = np.zeros(40)
    eta[[3, 17, 18]] = 1.0
    nref, ncoa = compare(d, eta, 0.5, 0.0, 3)
    assert nref == 3 and ncoa == 0


def test_plan_needs_room():
    from paper_2505_18743_amd.binding import load, make_mesh, SwAmrParams
    import ctypes
    from workloads.gen import uniform_mesh_desc
    d = uniform_mesh_desc(3, 3, 0.0, 0.0, 1.0)
    keep = []
    md = make_mesh(d, keep)
    eta = np.zeros(9)
    eta[4] = 1.0
    ap = SwAmrParams(0, 0.5, 0.0, 3, 0.0)
    n = ctypes.c_int32(0)
    st = load().sw_amr_plan(ctypes.byref(md), eta.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ap), 5,
                            ctypes.byref(n), None, None, None, None, None, None, None)
    assert st != 0 and n.value == 12
    assert b"cap" in load().sw_last_error()
