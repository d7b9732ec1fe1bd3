"""GPU adjoint: the HIP vector-Jacobian products against the oracle's reverse
mode (torch autograd through the oracle's residual and all-wet step), and the
checkpointed observation gradient against the oracle and central differences.
"""
import numpy as np
import pytest
import torch

from helpers import build_oracle
from oracle.adjoint import adjoint_gradients, allwet_step, point_operator, residual_vjp
from test_gpu_parity import gpu_from_oracle, hanging_case
from workloads import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(g, r):
    g = np.asarray(g).ravel()
    r = np.asarray(r).ravel()
    scale = np.abs(r).max()
    return np.abs(g - r).max() / (scale if scale > 0 else 1.0)


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("case", ["coastal_wet_dry", "hanging_elev"])
def test_vjp_operator_matches_oracle(case):
    say(f"case: vjp_operator {case}")
    rng = np.random.default_rng(5)
    if case == "coastal_wet_dry":
        wl = workload("coastal_steps_16")
        o, b = build_oracle(wl)
    else:
        o, b = hanging_case(r=2, S=(16, 8), tracer=False)
    K, NP = o.m.K, o.np_
    o.set_manning(rng.uniform(0.01, 0.04, K))
    o.set_bed_offset(rng.uniform(-0.02, 0.02, K))
    s = gpu_from_oracle(o, b)
    s.set_bed_offset(o.dbed.numpy())
    st = o.get_state()
    st = [st[0] + rng.uniform(-0.05, 0.05, st[0].shape), rng.uniform(-0.5, 0.5, st[0].shape),
          rng.uniform(-0.5, 0.5, st[0].shape)]
    bars = [rng.standard_normal((K, NP)) for _ in range(3)]
    t = 700.0
    ref = residual_vjp(o, st, t, *bars, o.nman.numpy(), o.dbed.numpy())
    got = s.vjp_operator(st[0], st[1], st[2], bars[0], bars[1], bars[2], t)
    s.sync()
    for name, g_, r_ in zip(("eta_b", "qx_b", "qy_b", "n_bar", "db_bar"), got, ref):
        e = rel(cpu(g_).reshape(r_.shape), r_)
        say(f"  {name} rel err {e:.3e}")
        assert e < 1e-12, (name, e)


def adjoint_small(n=8):
    wl = workload("adjoint_128", n=n)
    o, b = build_oracle(wl)
    _, _, _, _, dtb = o.residual(o.state, 0.0)
    dt = 0.9 * o.p.cfl * float(dtb)
    return wl, o, b, dt


def test_vjp_step_matches_oracle():
    say("case: vjp_step, one SSP3 step, 8x8 adjoint case")
    wl, o, b, dt = adjoint_small(8)
    K, NP = o.m.K, o.np_
    rng = np.random.default_rng(9)
    o.set_manning(rng.uniform(0.015, 0.04, K))
    o.set_bed_offset(np.where((o.m.ii + o.m.jj) % 2 == 1, 1e-3, -1e-3))
    dxy = o.dof_coords()
    L = o.m.nx0 * o.m.dx0
    st0 = [o.state[0].clone(), torch.as_tensor(np.sin(2 * np.pi * dxy[..., 1] / L)),
           torch.as_tensor(0.7 * np.cos(2 * np.pi * dxy[..., 0] / L))]
    t0 = 30.0
    # oracle: autograd through one all-wet step
    x = [v.clone().requires_grad_(True) for v in st0]
    n = o.nman.clone().requires_grad_(True)
    d = o.dbed.clone().requires_grad_(True)
    new, _ = allwet_step(o, x, t0, dt, d, n)
    w = [torch.as_tensor(rng.standard_normal((K, NP))) for _ in range(3)]
    obj = sum((new[f] * w[f]).sum() for f in range(3))
    gr = torch.autograd.grad(obj, x + [n, d])
    # GPU
    s = gpu_from_oracle(o, b)
    s.set_bed_offset(o.dbed.numpy())
    s.set_state(*[v.numpy() for v in st0])
    s.set_time(t0)
    stages = torch.empty(3, 3, s.n_dofs, dtype=torch.float64, device="cuda:0")
    s.step_record(dt, stages)
    sbar = torch.stack([torch.as_tensor(v.numpy().ravel()) for v in w], 0).to("cuda:0").contiguous()
    nbar = torch.zeros(K, dtype=torch.float64, device="cuda:0")
    dbar = torch.zeros(K, dtype=torch.float64, device="cuda:0")
    s.vjp_step(stages, t0, dt, sbar, nbar, dbar)
    s.sync()
    # the recorded forward equals the oracle's step
    e = rel(cpu(s.get_state()[0]).reshape(K, NP), new[0].detach().numpy())
    say(f"  forward zeta rel err {e:.3e}")
    assert e < 1e-11
    for name, g_, r_ in (("eta_b", sbar[0], gr[0]), ("qx_b", sbar[1], gr[1]), ("qy_b", sbar[2], gr[2]),
                         ("n_bar", nbar, gr[3]), ("db_bar", dbar, gr[4])):
        e = rel(cpu(g_).reshape(r_.shape), r_.numpy())
        say(f"  {name} rel err {e:.3e}")
        assert e < 1e-11, (name, e)


def test_observed_run_gradients_match_oracle():
    say("case: checkpointed observation gradient, 12x12 adjoint case, 11 steps, checkpoints every 4")
    from paper_2505_18743_amd.adjoint import PointObservation, observed_run
    wl, o, b, dt = adjoint_small(12)
    K, NP = o.m.K, o.np_
    rng = np.random.default_rng(21)
    L = o.m.nx0 * o.m.dx0
    gauges = rng.uniform(0.1 * L, 0.9 * L, size=(10, 2))
    cells, phi = point_operator(o, gauges)
    nsteps = 11
    s_ = gpu_from_oracle(o, b)
    gc, gp = s_.locate_points(gauges)
    assert np.array_equal(gc, cells) and np.abs(gp - phi).max() < 1e-14
    s_.close()
    st0 = [x.clone() for x in o.state[:3]]
    truth = np.zeros((nsteps, len(gauges)))
    n0 = np.full(K, 0.0275) + rng.uniform(-0.005, 0.005, K)
    d0 = np.where((o.m.ii + o.m.jj) % 2 == 1, 1e-3, -1e-3)
    loss_ref, gn_ref, gd_ref = adjoint_gradients(o, st0, 0.0, dt, nsteps, cells, phi, truth, n0, d0)
    s = gpu_from_oracle(o, b)
    obs = PointObservation(cells, phi, NP, "cuda:0")
    nman = torch.as_tensor(n0, device="cuda:0").requires_grad_(True)
    dbed = torch.as_tensor(d0, device="cuda:0").requires_grad_(True)
    state0 = [torch.as_tensor(v.numpy().ravel(), device="cuda:0") for v in st0]
    out = observed_run(s, nman, dbed, state0, 0.0, dt, nsteps, obs, checkpoint_every=4)
    loss = ((out - torch.as_tensor(truth, device="cuda:0")) ** 2).sum()
    loss.backward()
    s.sync()
    say(f"  loss {float(loss):.12e} oracle {loss_ref:.12e}")
    assert float(loss) == pytest.approx(loss_ref, rel=1e-11)
    en, ed = rel(cpu(nman.grad), gn_ref), rel(cpu(dbed.grad), gd_ref)
    say(f"  dL/dn rel err {en:.3e}  dL/ddb rel err {ed:.3e}")
    assert en < 1e-10 and ed < 1e-10


@pytest.mark.slow
def test_adjoint_128_full_size_central_differences():
    say("case: adjoint_128 full size, 200 steps, checkpoints every 20, gradient vs central differences")
    import time
    from paper_2505_18743_amd import Solver
    from paper_2505_18743_amd.adjoint import PointObservation, observed_run
    wl = workload("adjoint_128")
    s = Solver(wl["mesh"], wl["params"], "cuda:0")
    xy = s.node_coords()
    s.set_bathymetry(wl["bed"](xy[:, 0], xy[:, 1]))
    dof = s.dof_coords()
    eta0 = wl["eta0"](dof[:, 0], dof[:, 1])
    s.init_lake_at_rest(eta0)
    st = s.get_state()
    state0 = [x.clone() for x in st[:3]]
    K, NP = s.n_cells, s.np_
    dtb = s.apply_operator(*state0)[4]
    dt = 0.9 * float(dtb.cpu()[0])      # fixed: 0.9 x the positivity bound at t = 0
    cells, phi = s.locate_points(wl["gauges"])
    obs = PointObservation(cells, phi, NP, "cuda:0")
    nsteps = wl["steps"]
    truth = observed_run(s, torch.as_tensor(wl["manning_truth"], device="cuda:0"),
                         torch.zeros(K, dtype=torch.float64, device="cuda:0"), state0, 0.0, dt, nsteps, obs).detach()
    rng = np.random.default_rng(4)
    n0 = torch.full((K,), 0.0275, dtype=torch.float64, device="cuda:0")
    d0 = torch.as_tensor(np.where((np.arange(K) % 128 + np.arange(K) // 128) % 2 == 1, 1e-3, -1e-3),
                         device="cuda:0")
    # two losses: the gauge misfit against the truth run, and the squared free
    # surface at the gauges (O(1), so that central differences resolve it well)
    for lname, ref in (("misfit", truth), ("squared", torch.zeros_like(truth))):
        nman = n0.clone().requires_grad_(True)
        dbed = d0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = observed_run(s, nman, dbed, state0, 0.0, dt, nsteps, obs, checkpoint_every=20)
        loss = ((out - ref) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.sync()
        say(f"  {lname}: loss {float(loss):.6e}  forward {t1 - t0:.3f} s  backward {t2 - t1:.3f} s  "
            f"ratio {(t2 - t1) / (t1 - t0):.2f}")

        def L(n_, d_):
            with torch.no_grad():
                o_ = observed_run(s, n_, d_, state0, 0.0, dt, nsteps, obs)
                return float(((o_ - ref) ** 2).sum())

        h = 1e-6
        for trial in range(2):
            vn = torch.as_tensor(rng.standard_normal(K), device="cuda:0") * (trial != 1)
            vd = torch.as_tensor(rng.standard_normal(K), device="cuda:0") * (trial != 0)
            fd = (L(n0 + h * vn, d0 + h * vd) - L(n0 - h * vn, d0 - h * vd)) / (2 * h)
            ad = float((nman.grad * vn).sum() + (dbed.grad * vd).sum())
            say(f"  {lname} direction {trial}: FD {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(ad):.2e}")
            assert abs(fd - ad) <= (1e-5 if lname == "squared" else 1e-2) * abs(ad)
