"""The strong-friction channel of Sec. 4.3 (Table of channel parameters,
"strong friction" row): L = 100 m, q0 = 5 m^2/s, z_b0 = 4.5 m, c0 = 20 m,
Manning n = 1, a cos^4 bump in the depth profile, the given discharge at the
inflow, zeta = 0 at the outflow, walls north and south.

`steady_profile` integrates the steady-flow ODE eq:const_discharge,
(q0^2/(g h^3) - 1) dh/dx = -dz_b/dx + gamma(q0, h) q0 / (g h), with
gamma q0 / (g h) = n^2 q0^2 / h^(10/3), from h(L) = z_b(L) (zeta = 0) back
to x = 0 with the classical RK4 scheme on a fine grid, as the paper does for
its reference solution.
"""
import numpy as np

L, Q0, ZB0, C0, N_MAN, G = 100.0, 5.0, 4.5, 20.0, 1.0, 9.81


def depth(x):
    """z_b(x): depth of the bed below the datum (h = zeta + z_b)."""
    x = np.asarray(x, dtype=np.float64)
    s = x - L / 2
    return 4.9 + 0.001 * x - np.where(np.abs(s) <= C0, ZB0 * np.cos(np.pi * s / (2 * C0)) ** 4, 0.0)


def depth_dx(x):
    s = x - L / 2
    a = np.pi / (2 * C0)
    return 0.001 + np.where(np.abs(s) <= C0, 4 * ZB0 * a * np.cos(a * s) ** 3 * np.sin(a * s), 0.0)


def steady_profile(m=20000):
    """(x, zeta) of the steady state on m + 1 points, x ascending."""
    def f(x, h):
        return (-depth_dx(x) + N_MAN ** 2 * Q0 ** 2 / h ** (10.0 / 3.0)) / (Q0 ** 2 / (G * h ** 3) - 1.0)
    xs = np.linspace(L, 0.0, m + 1)
    h = np.empty_like(xs)
    h[0] = depth(L)
    for i in range(m):
        x, dx = xs[i], xs[i + 1] - xs[i]
        k1 = f(x, h[i])
        k2 = f(x + dx / 2, h[i] + dx / 2 * k1)
        k3 = f(x + dx / 2, h[i] + dx / 2 * k2)
        k4 = f(x + dx, h[i] + dx * k3)
        h[i + 1] = h[i] + dx / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return xs[::-1].copy(), (h - depth(xs))[::-1].copy()


def inflow(x, y):
    return np.zeros_like(x), np.full_like(x, Q0), np.zeros_like(x), np.zeros_like(x)


def channel_oracle(N, r, rk):
    """Oracle on N x 1 cells, GLL rule with r + 2 nodes, at rest (zeta = 0,
    q = q0); returns (oracle, bed elevation at the node coordinates)."""
    from oracle import Mesh, Oracle, Params
    m = Mesh.uniform(N, 1, 0.0, 0.0, L / N, bc=("discharge", "elev", "wall", "wall"))
    p = Params(r=r, S=(r + 2,), rule="gll", rk=rk, eps=1e-3, h_lim=1e-3, cfl=0.9, cfl_mode=1,
               tide=(0.0, 1.0, 0.0, 0.0), adapt_degree=False)
    o = Oracle(m, p)
    b = -depth(o.node_coords()[:, 0])
    o.set_bathymetry(b)
    o.set_manning(np.full(m.K, N_MAN))
    o.set_boundary_state(inflow)
    d = o.dof_coords()
    o.set_state(np.zeros(d.shape[:2]), np.full(d.shape[:2], Q0), np.zeros(d.shape[:2]))
    return o, b
