"""Closed-form solutions used to pin the oracle (test fixtures only)."""
from __future__ import annotations

import math

import numpy as np

G = 9.81


# ---- travelling vortex (Sec. 4.4) -----------------------------------------

def vortex_H(x):
    """The auxiliary function H(x) of the travelling-vortex depth profile (Sec. 4.4)."""
    c, s = np.cos(x), np.sin(x)
    c2x, s2x = np.cos(2 * x), np.sin(2 * x)
    return (35 * c2x / 384 + 35 * x * s2x / 192 + c ** 6 * (c ** 2 / 64 + 7 / 288)
            + 35 * c2x ** 2 / 3072 + 35 * x ** 2 / 256 + 35 * x * c2x * s2x / 768
            + x * c ** 5 * s * (c ** 2 + 7 / 6) / 8)


class Vortex:
    """Compact travelling vortex: h0=1, hmin=0.9, u_inf=6, r0=0.25, centre (0.5, 0.5)."""

    def __init__(self, h0=1.0, hmin=0.9, uinf=6.0, r0=0.25, x0=0.5, y0=0.5, g=G):
        self.h0, self.hmin, self.uinf, self.r0, self.x0, self.y0, self.g = h0, hmin, uinf, r0, x0, y0, g
        # Gamma such that h(0) = hmin
        dH = vortex_H(math.pi / 2) - vortex_H(0.0)
        self.Gamma = (math.pi / (4 * r0)) * math.sqrt(g * (h0 - hmin) / (4 * dH))

    def fields(self, x, y, t, period_x=None):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        cx = self.x0 + self.uinf * t
        dxv = x - cx
        if period_x is not None:
            dxv = (dxv + period_x / 2) % period_x - period_x / 2
        dyv = y - self.y0
        R = np.sqrt(dxv ** 2 + dyv ** 2)
        rho = math.pi * R / self.r0
        inside = rho < math.pi
        k = (4.0 / self.g) * (4 * self.Gamma * self.r0 / math.pi) ** 2
        h = np.where(inside, self.h0 - k * (vortex_H(math.pi / 2) - vortex_H(rho / 2)), self.h0)
        om = np.where(inside, 4 * self.Gamma * np.cos(rho / 2) ** 4, 0.0)
        u = self.uinf - dyv * om
        v = dxv * om
        return h, u, v


# ---- Ritter dam break on a flat dry bed --------------------------------------

def ritter(x, t, h0, xd, g=G):
    """Depth and velocity of the dam break onto a dry flat bed (Riemann invariants)."""
    x = np.asarray(x, dtype=np.float64)
    c0 = math.sqrt(g * h0)
    xi = (x - xd) / t
    h = np.where(xi <= -c0, h0, np.where(xi < 2 * c0, (2 * c0 - xi) ** 2 / (9 * g), 0.0))
    u = np.where(xi <= -c0, 0.0, np.where(xi < 2 * c0, 2.0 / 3.0 * (xi + c0), 0.0))
    return h, u


# ---- uniform flow decaying under Manning friction -----------------------------

def manning_decay(q0, h, n, t, g=G):
    """|q|(t) for dq/dt = -g n^2 |q| q / h^{7/3} with h fixed."""
    k = g * n * n / h ** (7.0 / 3.0)
    return q0 / (1.0 + k * q0 * t)


# ---- Thacker's radially symmetric paraboloid (Sec. 4.3) -------------------------

class Thacker:
    def __init__(self, h0=0.1, L=3.0, a=1.0, r0=0.8, g=G):
        self.h0, self.L, self.a, self.r0, self.g = h0, L, a, r0, g
        self.omega = math.sqrt(8 * g * h0) / a
        self.A = (a * a - r0 * r0) / (a * a + r0 * r0)

    def depth_bed(self, x, y):
        """Bathymetry depth z_b(R) = h0 (1 - R^2/a^2) (positive = below datum)."""
        R2 = (np.asarray(x) - self.L / 2) ** 2 + (np.asarray(y) - self.L / 2) ** 2
        return self.h0 * (1 - R2 / self.a ** 2)

    def zeta(self, x, y, t):
        R2 = (np.asarray(x) - self.L / 2) ** 2 + (np.asarray(y) - self.L / 2) ** 2
        A, w = self.A, self.omega
        f = math.sqrt(1 - A * A) / (1 - A * math.cos(w * t))
        return -self.h0 * (f - 1 - R2 / self.a ** 2 * (f * f - 1))
