"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only input data: point sets, workload parameters and seeded
test vectors.  It contains none of the method's arithmetic (no tree, no
sampling, no factorisation, no Hessian application) and imports neither the
oracle nor the HIP library.

Workloads (sizes follow the paper's experiments: 1D with leaf 32, 2D grids with
leaf 64, eps = 1e-4; Sec. 4.1, 4.2 and Appendix A):
  kernel1d      N points at cell centres of [0,1]; H = exp(-|x-y|/ell) + shift I
  diffusion2d   Gauss-Newton Hessian of an initial-condition inversion for
                explicit-Euler heat flow on an n x n interior grid
  kernel2d      N = nx*ny cell centres of a grid; H = exp(-r/ell) + shift I
  batch         256 uneven 2D kernel problems on random-aspect grids
  advdiff2d     misfit Gauss-Newton Hessian of upwind advection-diffusion
  minsurf2d     Hessian of the discrete minimal-surface area at a smooth surface
                (two successive surfaces, as two steps of an optimisation)
"""
import math

import numpy as np


# ---------------------------------------------------------------- point sets
def points_1d_cell_centres(n):
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def points_grid_interior(n):
    """Interior nodes ((ix+1)h, (iy+1)h), h = 1/(n+1); user index iy*n + ix."""
    h = 1.0 / (n + 1)
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([(ix.ravel() + 1) * h, (iy.ravel() + 1) * h], axis=1)


def points_grid_cell_centres(nx, ny, h=None):
    """Cell centres ((ix+0.5)h, (iy+0.5)h); user index iy*nx + ix."""
    if h is None:
        h = 1.0 / max(nx, ny)
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(ix.ravel() + 0.5) * h, (iy.ravel() + 0.5) * h], axis=1)


def gaussian_vectors(n, nv, seed):
    """Seeded N(0,1) test vectors (user order), float64, shape (n, nv)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((n, nv))


# ---------------------------------------------------------------- workloads
def config_kernel1d(n=1024):
    return dict(name="kernel1d", n=n, points=points_1d_cell_centres(n), ell=0.1,
                shift=1e-2, leaf=32, eta=0.7, cap=16, p=10, adaptive=False,
                tol=1e-4, seed=1, vec_seed=101, nv=16, ns_iters=20)


def diffusion_obs_index(n, count=10):
    """0-based observation indices per axis: equispaced interior nodes.

    For n = 64 and count = 10 this is 1-based round(6.5 j + 3.25), j = 0..9.
    """
    step = (n + 1) / count
    return np.array([int(math.floor(step * j + step / 2 + 0.5)) - 1 for j in range(count)],
                    dtype=np.int64)


def config_diffusion2d(n=64):
    h = 1.0 / (n + 1)
    return dict(name="diffusion2d", grid=n, n=n * n, points=points_grid_interior(n), h=h,
                kappa=1e-2, dt=4.5e-3, steps=100, obs_steps=list(range(80, 101, 5)),
                obs_index=diffusion_obs_index(n), sigma=1e-2, gamma=1e-2, beta=0.01,
                leaf=64, eta=0.7, cap=24, p=10, adaptive=True, tol=1e-4, seed=2)


def config_kernel2d(nside=256, ell=0.05, shift=1e-3):
    return dict(name="kernel2d", n=nside * nside, nx=nside, ny=nside,
                points=points_grid_cell_centres(nside, nside), ell=ell, shift=shift,
                leaf=64, eta=0.7, cap=32, p=10, adaptive=True, tol=1e-4, seed=3,
                vec_seed=303, nv=64)


def batch_problem(b, base_seed=4000):
    """Problem b of the uneven batch: N log-uniform in [1024, 16384]."""
    g = np.random.Generator(np.random.PCG64(base_seed + b))
    n_target = int(round(math.exp(g.uniform(math.log(1024), math.log(16384)))))
    aspect = math.exp(g.uniform(math.log(0.25), math.log(4.0)))
    nx = max(8, int(round(math.sqrt(n_target * aspect))))
    ny = max(8, int(round(n_target / nx)))
    ell = g.uniform(0.02, 0.2)
    h = 1.0 / max(nx, ny)
    return dict(name="kernel2d", n=nx * ny, nx=nx, ny=ny, ell=ell, shift=1e-3,
                points=points_grid_cell_centres(nx, ny, h), leaf=64, eta=0.7, cap=32,
                p=10, adaptive=True, tol=1e-4, seed=base_seed + b)


def config_batch(count=256):
    return [batch_problem(b) for b in range(count)]


def advdiff_velocity_modes(seed=5, modes=4):
    g = np.random.Generator(np.random.PCG64(seed))
    a = g.integers(1, 5, size=modes)
    b = g.integers(1, 5, size=modes)
    s = g.choice(np.array([-1.0, 1.0]), size=modes)
    return a.astype(np.int64), b.astype(np.int64), s


def config_advdiff2d(n=128, nobs=400, obs_seed=55, vel_seed=5):
    h = 1.0 / (n + 1)
    a, b, s = advdiff_velocity_modes(vel_seed)
    obs = np.random.Generator(np.random.PCG64(obs_seed)).uniform(0.0, 1.0, size=(nobs, 2))
    return dict(name="advdiff2d", grid=n, n=n * n, points=points_grid_interior(n), h=h,
                kappa=1e-3, steps=400, obs_steps=list(range(40, 401, 40)), obs_points=obs,
                sigma=1e-2, mode_a=a, mode_b=b, mode_s=s, leaf=64, eta=0.7, cap=32, p=10,
                adaptive=True, tol=1e-4, seed=6)


def learned_training_problem(i, base_seed=10000):
    """Problem i of the rank-predictor training set: even i from the 1D
    kernel family (N log-uniform in [512, 4096] cell centres, ell ~ U[0.02,
    0.3], shift 10^U[-3, -1], leaf 32, cap 16), odd i from the 2D grid family
    (side 32..128, ell ~ U[0.02, 0.2], shift 10^U[-3, -2], leaf 64, cap 32);
    eps drawn from {1e-3, 1e-4, 1e-5, 1e-6}."""
    g = np.random.Generator(np.random.PCG64(base_seed + i))
    eps = float(g.choice([1e-3, 1e-4, 1e-5, 1e-6]))
    if i % 2 == 0:
        n = int(round(math.exp(g.uniform(math.log(512), math.log(4096)))))
        return dict(name="kernel1d", n=n, points=points_1d_cell_centres(n),
                    ell=float(g.uniform(0.02, 0.3)), shift=float(10 ** g.uniform(-3, -1)),
                    leaf=32, eta=0.7, cap=16, p=10, tol=eps, seed=base_seed + i)
    side = int(g.integers(32, 129))
    return dict(name="kernel2d", n=side * side, points=points_grid_cell_centres(side, side),
                ell=float(g.uniform(0.02, 0.2)), shift=float(10 ** g.uniform(-3, -2)),
                leaf=64, eta=0.7, cap=32, p=10, tol=eps, seed=base_seed + i)


def minsurf_heights(n, step=0):
    """Node heights ((n+2) x (n+2), [iy, ix], boundary included) of a smooth
    synthetic surface over the unit square, spacing h = 1/(n+1): a saddle
    frame (x-1/2)^2 - (y-1/2)^2 on the boundary with an interior bump
    0.1 sin(pi x) sin(2 pi y); step 1 adds an interior change
    0.05 sin(2 pi x) sin(pi y), standing in for the next iterate of an
    optimisation (the boundary stays fixed)."""
    t = np.arange(n + 2, dtype=np.float64) / (n + 1)
    Y, X = np.meshgrid(t, t, indexing="ij")
    M = (X - 0.5) ** 2 - (Y - 0.5) ** 2 + 0.1 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    if step >= 1:
        M = M + 0.05 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    return M


def config_minsurf2d(n=128, step=0):
    return dict(name="minsurf2d", grid=n, n=n * n, points=points_grid_interior(n),
                heights=minsurf_heights(n, step), leaf=64, eta=0.7, cap=32, p=10,
                adaptive=True, tol=1e-6, seed=7, eps=1e-4, eps_build=1e-6)
