"""GPU: sw_apply_operator_noalloc (the operator evaluation whose scratch lives
in the library's fixed device array) against sw_apply_operator, through the
C ABI: two calls in a row, the second on a smaller context (the array keeps
the first call's contents), then a context too large for the array, which
the entry point refuses before launching anything."""
import numpy as np
import pytest
import torch

from test_gpu_parity import TOL_RHS, cpu, gpu_from_oracle, hanging_case, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def both(s, st, t):
    ref = s.apply_operator(st[0], st[1], st[2], st[3], t)
    out = [torch.full((s.n_dofs,), np.nan, dtype=torch.float64, device=s.dev) for _ in range(4)]
    out.append(torch.full((1,), np.nan, dtype=torch.float64, device=s.dev))
    s.apply_operator_noalloc(st[0], st[1], st[2], st[3], t, out)
    s.sync()
    return ref, out


def test_noalloc_operator_matches_and_shrinks():
    rng = np.random.default_rng(3)
    cases = [("hanging r=3 S=(16,8,5), tracer, tide", hanging_case(3, (16, 8, 5))),
             ("hanging r=1 S=(8,4), tracer, tide (smaller)", hanging_case(1, (8, 4)))]
    sizes = []
    for label, (o, b) in cases:
        s = gpu_from_oracle(o, b)
        K = o.m.K
        say(f"case: {label}, {K} cells, {s.n_dofs} dofs per field")
        st0 = o.get_state()
        st = [st0[0], rng.uniform(-0.5, 0.5, st0[0].shape), rng.uniform(-0.5, 0.5, st0[0].shape), st0[3]]
        ref, out = both(s, st, 700.0)
        for name, a, r_ in (("F", out[0], ref[0]), ("Gx", out[1], ref[1]), ("Gy", out[2], ref[2]),
                            ("R", out[3], ref[3])):
            e = rel(cpu(a, K), cpu(r_, K))
            say(f"  {name} rel diff {e:.3e}")
            assert e < TOL_RHS and torch.equal(a, r_), (label, name, e)
        assert torch.equal(out[4], ref[4]), (label, float(out[4][0]), float(ref[4][0]))
        # the oracle too
        F, Gx, Gy, R, dtb = o.apply_operator(st, 700.0)
        for name, a, r_ in (("F", out[0], F), ("Gx", out[1], Gx), ("Gy", out[2], Gy), ("R", out[3], R)):
            assert rel(cpu(a, K), r_) < TOL_RHS, (label, name)
        assert float(out[4][0]) == pytest.approx(dtb, rel=1e-12)
        sizes.append(s.n_dofs)
        s.close()
    assert sizes[1] < sizes[0]


def test_noalloc_operator_refuses_a_context_above_its_scratch():
    from paper_2505_18743_amd import Solver
    from workloads import uniform_mesh_desc
    n = 420                     # 176,400 cells, r = 2: 4 x 1.59 M residual doubles > 6 Mi
    say(f"case: {n}x{n} r=2 context, scratch size check")
    mesh = uniform_mesh_desc(n, n, 0.0, 0.0, 10.0)
    params = dict(r=2, S=(4,), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1, eps0=1e-8, newton_max=20,
                  cfl=0.9, cfl_mode=1, tracer=False, tide=(0.0, 1.0, 0.0, 0.0))
    s = Solver(mesh, params, device="cuda:0")
    s.set_bathymetry(torch.full((s.n_vol,), -5.0, dtype=torch.float64, device=s.dev))
    z = s.zeros()
    out = [s.zeros() for _ in range(3)] + [None, None]
    with pytest.raises(RuntimeError, match="status -1.*doubles of device scratch"):
        s.apply_operator_noalloc(z, z, z, None, 0.0, out)
    s.close()
