"""Seeded synthetic workloads with the shapes of the paper's coastal cases.

Every random draw comes from ``numpy.random.Generator(PCG64(seed))``.  The
bathymetry is a raster with bilinear interpolation inside each pixel, as the
paper does with its 30 m lagoon dataset (Sec. 5); callers sample it at the
quadrature-node coordinates their own code computes.

Workloads (sizes are the ones the benchmarks and parity tests use):

  coastal_steps_16   16x16 cells on 1 km^2, r=1, 8x8 samples: random
                     piecewise-constant steps in [-5,-1] m on a 12x12 patch
                     grid plus three 2 m Gaussian bumps (sigma 100 m); lake at
                     rest plus a 0.1 m Gaussian hump (sigma 150 m); walls;
                     SSP3 at CFL 0.2; 100 steps.
  beach_dambreak_256 256x256 cells on 20 km^2, r=2, 16x16 samples: linear
                     beach -10 m .. +2 m, fractal noise (spectral slope -3,
                     rms 0.5 m), three cross-shore channel cuts (150 m wide,
                     2 m deep, discontinuous edges); dam break eta = 1 m for
                     x < 10 km, 0 elsewhere; Manning 0.025; walls; 500 steps.
  tidal_quadtree_r3  128x128 coarse 200 m cells refined twice where the
                     bathymetry range is largest (about 100k leaves, 2:1
                     balanced), r=3, 32/16/8 samples per level, fractal bed in
                     [-30,+3] m, 0.5 m tide (period 44712 s) on the west side,
                     Gaussian tracer, Manning 0.025; SSP3 at 0.4 of the
                     positivity bound; 1000 steps.
  adjoint_128        128x128 cells of 100 m, r=2, 16x16 samples, fractal bed
                     in [-20,-2] m, 16 Gaussian humps, 64 gauges, truth Manning
                     U[0.015,0.04]; 200 steps.
  ensemble_64        64 members, N ~ U{32..256}, r ~ U{1,2,3}, 16x16 samples,
                     fractal bed in [-15,+2] m, west tide amplitude U[0.2,1],
                     Manning U[0.015,0.035]; 300 steps.
"""
from __future__ import annotations

import numpy as np

SEED0 = 2505187430


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


class Raster:
    """Values on a regular grid; bilinear interpolation inside each pixel."""

    def __init__(self, x0, y0, spacing, values):
        self.x0, self.y0, self.h = float(x0), float(y0), float(spacing)
        self.v = np.ascontiguousarray(values, dtype=np.float64)   # [ny, nx]

    def sample(self, x, y):
        if type(x).__module__.startswith("torch"):
            return self._sample_torch(x, y)
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        ny, nx = self.v.shape
        fx = np.clip((x - self.x0) / self.h, 0.0, nx - 1.0)
        fy = np.clip((y - self.y0) / self.h, 0.0, ny - 1.0)
        i = np.minimum(fx.astype(np.int64), nx - 2)
        j = np.minimum(fy.astype(np.int64), ny - 2)
        tx, ty = fx - i, fy - j
        v = self.v
        return ((1 - ty) * ((1 - tx) * v[j, i] + tx * v[j, i + 1])
                + ty * ((1 - tx) * v[j + 1, i] + tx * v[j + 1, i + 1]))

    def _sample_torch(self, x, y):
        """The same interpolation on torch tensors (any device)."""
        import torch
        v = torch.as_tensor(self.v, device=x.device)
        ny, nx = self.v.shape
        fx = ((x - self.x0) / self.h).clamp(0.0, nx - 1.0)
        fy = ((y - self.y0) / self.h).clamp(0.0, ny - 1.0)
        i = fx.to(torch.int64).clamp(max=nx - 2)
        j = fy.to(torch.int64).clamp(max=ny - 2)
        tx, ty = fx - i, fy - j
        return ((1 - ty) * ((1 - tx) * v[j, i] + tx * v[j, i + 1])
                + ty * ((1 - tx) * v[j + 1, i] + tx * v[j + 1, i + 1]))

    def cell_range(self, x0, y0, dx):
        """(min, max) of the raster over the pixels touched by a square."""
        ny, nx = self.v.shape
        i0 = int(np.clip(np.floor((x0 - self.x0) / self.h), 0, nx - 1))
        i1 = int(np.clip(np.ceil((x0 + dx - self.x0) / self.h), 0, nx - 1))
        j0 = int(np.clip(np.floor((y0 - self.y0) / self.h), 0, ny - 1))
        j1 = int(np.clip(np.ceil((y0 + dx - self.y0) / self.h), 0, ny - 1))
        blk = self.v[j0:j1 + 1, i0:i1 + 1]
        return float(blk.min()), float(blk.max())


def fractal_raster(n, slope, rms, rng):
    """Gaussian random field on an n x n raster with isotropic PSD ~ |k|^slope,
    zero mean and the given rms (FFT synthesis)."""
    kx = np.fft.fftfreq(n)
    ky = np.fft.rfftfreq(n)
    kk = np.sqrt(kx[:, None] ** 2 + ky[None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (slope / 2.0)
    noise = rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)
    f = np.fft.irfft2(amp * noise, s=(n, n))
    f -= f.mean()
    f *= rms / f.std()
    return f


def uniform_mesh_desc(nx, ny, x0, y0, dx, bc=("wall",) * 4):
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return dict(nx0=nx, ny0=ny, x0=float(x0), y0=float(y0), dx0=float(dx),
                level=np.zeros(nx * ny, np.int32), i=ii.ravel().astype(np.int32),
                j=jj.ravel().astype(np.int32), bc=tuple(bc))


def quadtree_desc(nx0, ny0, x0, y0, dx0, refine_fn, nlev, bc=("wall",) * 4):
    """Quadtree leaves refined where ``refine_fn(level, x, y, dx, leaves)`` selects,
    then closed so neighbouring leaves differ by at most one level (2:1).
    Leaves are returned sorted by (level, j, i)."""
    leaves = {(0, i, j) for i in range(nx0) for j in range(ny0)}
    for L in range(nlev):
        cand = sorted(k for k in leaves if k[0] == L)
        pick = refine_fn(L, cand)
        for (lv, i, j) in pick:
            leaves.discard((lv, i, j))
            for a in (0, 1):
                for b in (0, 1):
                    leaves.add((lv + 1, 2 * i + a, 2 * j + b))
        # 2:1 closure
        changed = True
        while changed:
            changed = False
            for (lv, i, j) in sorted(leaves, key=lambda k: -k[0]):
                if (lv, i, j) not in leaves or lv < 2:
                    continue
                for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                    ni, nj = i + di, j + dj
                    if not (0 <= ni < nx0 << lv and 0 <= nj < ny0 << lv):
                        continue
                    # a leaf two levels coarser covering the neighbour position
                    ck = (lv - 2, ni >> 2, nj >> 2)
                    if ck in leaves:
                        leaves.discard(ck)
                        for a in (0, 1):
                            for b in (0, 1):
                                leaves.add((lv - 1, 2 * ck[1] + a, 2 * ck[2] + b))
                        changed = True
    order = sorted(leaves, key=lambda k: (k[0], k[2], k[1]))
    lev = np.array([k[0] for k in order], np.int32)
    ii = np.array([k[1] for k in order], np.int32)
    jj = np.array([k[2] for k in order], np.int32)
    return dict(nx0=nx0, ny0=ny0, x0=float(x0), y0=float(y0), dx0=float(dx0),
                level=lev, i=ii, j=jj, bc=tuple(bc))


def _gauss(x, y, cx, cy, sigma):
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sigma ** 2))


# ---------------------------------------------------------------------------

def _coastal_steps_16(seed, n=16):
    rng = _rng(seed)
    L = 1000.0
    patches = rng.uniform(-5.0, -1.0, size=(12, 12))
    centres = rng.uniform(0.0, L, size=(3, 2))

    def bed(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        pi = np.clip((x / (L / 12.0)).astype(np.int64), 0, 11)
        pj = np.clip((y / (L / 12.0)).astype(np.int64), 0, 11)
        b = patches[pj, pi].copy()
        for cx, cy in centres:
            b = b + 2.0 * _gauss(x, y, cx, cy, 100.0)
        return b

    def eta0(x, y):
        return 0.1 * _gauss(np.asarray(x), np.asarray(y), L / 2, L / 2, 150.0)

    mesh = uniform_mesh_desc(n, n, 0.0, 0.0, L / n)
    params = dict(r=1, S=(8,), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1,
                  eps0=1e-8, newton_max=20, cfl=0.2, cfl_mode=0, tracer=False,
                  tide=(0.0, 1.0, 0.0, 0.0))
    return dict(name="coastal_steps_16", mesh=mesh, params=params, bed=bed, eta0=eta0,
                lake_at_rest=True, manning=np.zeros(n * n), steps=100, tracer0=None)


def _beach_dambreak(seed, n=256, window=None):
    """Full 256x256 case; ``window=(i0, j0, nx, ny)`` gives a crop with the same
    cell size and bathymetry (used where the oracle must run many steps)."""
    rng = _rng(seed)
    L = 20000.0
    nr = 2049
    f = fractal_raster(nr - 1, -3.0, 0.5, rng)
    f = np.pad(f, ((0, 1), (0, 1)), mode="wrap")
    ras = Raster(0.0, 0.0, L / (nr - 1), f)
    cut_y = rng.uniform(1000.0, L - 1000.0, size=3)

    def bed(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        b = -10.0 + 12.0 * x / L + ras.sample(x, y)
        for cy in cut_y:
            b = np.where(np.abs(y - cy) < 75.0, b - 2.0, b)
        return b

    def eta0(x, y):
        return np.where(np.asarray(x) < 10000.0, 1.0, 0.0)

    dx = L / n
    if window is None:
        mesh = uniform_mesh_desc(n, n, 0.0, 0.0, dx)
    else:
        i0, j0, nx, ny = window
        mesh = uniform_mesh_desc(nx, ny, i0 * dx, j0 * dx, dx)
    K = mesh["level"].size
    params = dict(r=2, S=(16,), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1,
                  eps0=1e-8, newton_max=20, cfl=0.9, cfl_mode=1, tracer=False,
                  tide=(0.0, 1.0, 0.0, 0.0))
    return dict(name="beach_dambreak_256" if window is None else "beach_dambreak_crop",
                mesh=mesh, params=params, bed=bed, eta0=eta0, lake_at_rest=True,
                manning=np.full(K, 0.025), steps=500, tracer0=None, cut_y=cut_y)


def _tidal_quadtree(seed, nx0=128, target=100_000):
    rng = _rng(seed)
    dx0 = 200.0
    L = nx0 * dx0
    nr = 2049
    f = fractal_raster(nr - 1, -3.0, 1.0, rng)
    f = np.pad(f, ((0, 1), (0, 1)), mode="wrap")
    f = (f - f.min()) / (f.max() - f.min())
    ras = Raster(0.0, 0.0, L / (nr - 1), -30.0 + 33.0 * f)

    def refine_fn(level, cand):
        if not cand:
            return []
        rng_vals = np.array([np.subtract(*ras.cell_range(i * dx0 / 2 ** lv, j * dx0 / 2 ** lv,
                                                            dx0 / 2 ** lv)[::-1]) for (lv, i, j) in cand])
        frac = 0.55 if nx0 == 128 else 0.55
        k = int(round(frac * len(cand)))
        order = np.argsort(-rng_vals, kind="stable")
        return [cand[t] for t in order[:k]]

    mesh = quadtree_desc(nx0, nx0, 0.0, 0.0, dx0, refine_fn, 2, bc=("elev", "wall", "wall", "wall"))
    K = mesh["level"].size

    def bed(x, y):
        return ras.sample(x, y)

    def eta0(x, y):
        return np.zeros_like(np.asarray(x, dtype=np.float64))

    def tracer0(x, y):
        return _gauss(np.asarray(x), np.asarray(y), L / 2, L / 2, 2000.0)

    # dt = 0.4 x the positivity bound: on the finest level r = 3 meets the
    # 8-point equispaced rule, which is linearly unstable above about half
    # the bound (a 1e-6 m tide grows 2.5x per step at 0.9 and at 0.6, and
    # stays bounded at 0.5 and below)
    params = dict(r=3, S=(32, 16, 8), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1,
                  eps0=1e-8, newton_max=20, cfl=0.4, cfl_mode=1, tracer=True,
                  tide=(0.5, 44712.0, 0.0, 0.0))
    return dict(name="tidal_quadtree_r3", mesh=mesh, params=params, bed=bed, eta0=eta0,
                lake_at_rest=True, manning=np.full(K, 0.025), steps=1000, tracer0=tracer0)


def _adjoint_128(seed, n=128):
    rng = _rng(seed)
    dx = 100.0
    L = n * dx
    nr = 1025
    f = fractal_raster(nr - 1, -3.0, 1.0, rng)
    f = np.pad(f, ((0, 1), (0, 1)), mode="wrap")
    f = (f - f.min()) / (f.max() - f.min())
    ras = Raster(0.0, 0.0, L / (nr - 1), -20.0 + 18.0 * f)
    hump = rng.uniform(0.1 * L, 0.9 * L, size=(16, 2))
    gauges = rng.uniform(0.05 * L, 0.95 * L, size=(64, 2))
    n_truth = rng.uniform(0.015, 0.04, size=n * n)

    def bed(x, y):
        return ras.sample(x, y)

    def eta0(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        e = np.zeros_like(x)
        for cx, cy in hump:
            e = e + 0.2 * _gauss(x, y, cx, cy, 500.0)
        return e

    mesh = uniform_mesh_desc(n, n, 0.0, 0.0, dx)
    params = dict(r=2, S=(16,), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1,
                  eps0=1e-8, newton_max=20, cfl=0.9, cfl_mode=1, tracer=False,
                  tide=(0.0, 1.0, 0.0, 0.0))
    return dict(name="adjoint_128", mesh=mesh, params=params, bed=bed, eta0=eta0,
                lake_at_rest=True, manning=np.full(n * n, 0.0275), manning_truth=n_truth,
                gauges=gauges, steps=200, checkpoint_every=20, tracer0=None)


def _ensemble_64(seed, members=64, nmin=32, nmax=256):
    rng = _rng(seed)
    out = []
    for m in range(members):
        sub = _rng(seed * 1000 + m)
        N = int(rng.integers(nmin, nmax + 1))
        r = int(rng.integers(1, 4))
        A = float(rng.uniform(0.2, 1.0))
        nm = float(rng.uniform(0.015, 0.035))
        L = 20000.0
        nr = 1025
        f = fractal_raster(nr - 1, -3.0, 1.0, sub)
        f = np.pad(f, ((0, 1), (0, 1)), mode="wrap")
        f = (f - f.min()) / (f.max() - f.min())
        ras = Raster(0.0, 0.0, L / (nr - 1), -15.0 + 17.0 * f)
        mesh = uniform_mesh_desc(N, N, 0.0, 0.0, L / N, bc=("elev", "wall", "wall", "wall"))
        params = dict(r=r, S=(16,), rule="eq", rk="ssp3", g=9.81, eps=0.1, h_lim=0.1,
                      eps0=1e-8, newton_max=20, cfl=0.9, cfl_mode=1, tracer=False,
                      tide=(A, 44712.0, np.pi / 2, 0.0))
        out.append(dict(name=f"member{m}", mesh=mesh, params=params, bed=ras.sample,
                        eta0=lambda x, y: np.zeros_like(np.asarray(x, dtype=np.float64)),
                        lake_at_rest=True, manning=np.full(N * N, nm), steps=300, tracer0=None))
    return out


WORKLOADS = {
    "coastal_steps_16": lambda **kw: _coastal_steps_16(SEED0 + 0, **kw),
    "beach_dambreak_256": lambda **kw: _beach_dambreak(SEED0 + 1, **kw),
    "tidal_quadtree_r3": lambda **kw: _tidal_quadtree(SEED0 + 2, **kw),
    "adjoint_128": lambda **kw: _adjoint_128(SEED0 + 3, **kw),
    "ensemble_64": lambda **kw: _ensemble_64(SEED0 + 4, **kw),
}


def workload(name, **kw):
    return WORKLOADS[name](**kw)
