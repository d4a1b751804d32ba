"""Synthetic Hessian-vector products of the workloads (oracle side, float64).

These play the role of the user's PDE solver: the paper's Hessians are known
only through products with vectors, each costing a forward and an adjoint
solve (Sec. 2, the Hessian expression and the cost statement that follows it;
Sec. 3.3).  All apply to user-ordered columns V of shape (N, nv).

  KernelHessian      H_ij = exp(-|x_i - x_j| / ell) + shift delta_ij
  DiffusionGN        H = F^T F / sigma^2 + gamma (I - beta Lap)^2, where F maps an
                     initial condition through explicit-Euler heat steps to point
                     observations at several times; F^T by exact adjoint steps
  AdvDiffGN          H = F^T F / sigma^2 with first-order upwind advection-diffusion
                     and bilinear point observations (misfit only, as in Sec. 4.2)
  MinimalSurface     Hessian of the discrete minimal-surface area at a given surface
                     (Appendix A, the shape-optimisation example)
"""
import numpy as np


class KernelHessian:
    def __init__(self, points, ell, shift, chunk=2048):
        p = np.asarray(points, dtype=np.float64)
        self.p = p.reshape(len(p), -1)
        self.n = len(self.p)
        self.ell = float(ell)
        self.shift = float(shift)
        self.chunk = chunk

    def block(self, rows, cols):
        d = self.p[rows][:, None, :] - self.p[cols][None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        K = np.exp(-r / self.ell)
        K[np.asarray(rows)[:, None] == np.asarray(cols)[None, :]] += self.shift
        return K

    def dense(self):
        idx = np.arange(self.n)
        return self.block(idx, idx)

    def apply(self, V):
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        V = V.reshape(self.n, -1)
        out = np.empty_like(V)
        cols = np.arange(self.n)
        for a in range(0, self.n, self.chunk):
            rows = np.arange(a, min(self.n, a + self.chunk))
            out[rows] = self.block(rows, cols) @ V
        return out.ravel() if vec else out


def _lap(u, h):
    """5-point Laplacian with zero Dirichlet data; u has shape (ny, nx, nv)."""
    out = -4.0 * u
    out[1:] += u[:-1]
    out[:-1] += u[1:]
    out[:, 1:] += u[:, :-1]
    out[:, :-1] += u[:, 1:]
    return out / (h * h)


class DiffusionGN:
    """Initial-condition inversion for u_t = kappa Lap u (explicit Euler)."""

    def __init__(self, cfg):
        self.g = cfg["grid"]
        self.n = self.g * self.g
        self.h = cfg["h"]
        self.kappa = cfg["kappa"]
        self.dt = cfg["dt"]
        self.steps = cfg["steps"]
        self.obs_steps = set(cfg["obs_steps"])
        self.oi = np.asarray(cfg["obs_index"])
        self.sigma = cfg["sigma"]
        self.gamma = cfg["gamma"]
        self.beta = cfg["beta"]

    def step(self, u):
        return u + (self.dt * self.kappa) * _lap(u, self.h)

    def observe(self, u):
        return u[np.ix_(self.oi, self.oi)]

    def observe_T(self, d):
        out = np.zeros((self.g, self.g) + d.shape[2:])
        out[np.ix_(self.oi, self.oi)] = d
        return out

    def forward(self, V):
        """F V: observations at each observation step, list of (10, 10, nv)."""
        u = V.reshape(self.g, self.g, -1).copy()
        obs = []
        for s in range(1, self.steps + 1):
            u = self.step(u)
            if s in self.obs_steps:
                obs.append(self.observe(u))
        return obs

    def adjoint(self, obs):
        """F^T applied to a list of observation arrays (one per observation step)."""
        nv = obs[0].shape[2]
        lam = np.zeros((self.g, self.g, nv))
        times = sorted(self.obs_steps)
        for s in range(self.steps, 0, -1):
            if s in self.obs_steps:
                lam = lam + self.observe_T(obs[times.index(s)])
            lam = self.step(lam)       # the step operator is symmetric
        return lam.reshape(self.n, nv)

    def regularization(self, V):
        u = V.reshape(self.g, self.g, -1)
        r = u - self.beta * _lap(u, self.h)
        r = r - self.beta * _lap(r, self.h)
        return self.gamma * r.reshape(self.n, -1)

    def apply(self, V):
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        V = V.reshape(self.n, -1)
        out = self.adjoint(self.forward(V)) / (self.sigma * self.sigma) + self.regularization(V)
        return out.ravel() if vec else out


class AdvDiffGN:
    """Misfit Gauss-Newton Hessian of u_t + v.grad u = kappa Lap u (upwind Euler)."""

    def __init__(self, cfg):
        self.g = cfg["grid"]
        self.n = self.g * self.g
        self.h = cfg["h"]
        self.kappa = cfg["kappa"]
        self.steps = cfg["steps"]
        self.obs_steps = list(cfg["obs_steps"])
        self.sigma = cfg["sigma"]
        g, h = self.g, self.h
        x = (np.arange(g) + 1) * h
        X, Y = np.meshgrid(x, x, indexing="xy")   # X[iy, ix] = x, Y[iy, ix] = y
        vx = np.zeros_like(X)
        vy = np.zeros_like(X)
        for a, b, s in zip(cfg["mode_a"], cfg["mode_b"], cfg["mode_s"]):
            # psi = s sin(pi a x) sin(pi b y);  v = (d psi/dy, -d psi/dx)
            vx += s * np.sin(np.pi * a * X) * np.pi * b * np.cos(np.pi * b * Y)
            vy -= s * np.pi * a * np.cos(np.pi * a * X) * np.sin(np.pi * b * Y)
        self.vx, self.vy = vx, vy
        vmax = float(np.max(np.abs(vx) + np.abs(vy)))
        self.dt = 0.5 * min(h / vmax, h * h / (4.0 * self.kappa))
        # bilinear observation weights on interior nodes (boundary values are zero)
        pts = np.asarray(cfg["obs_points"])
        rows, cols, vals = [], [], []
        for q, (px, py) in enumerate(pts):
            fx, fy = px / h, py / h
            i0, j0 = int(np.floor(fx)), int(np.floor(fy))
            tx, ty = fx - i0, fy - j0
            for di, wx in ((0, 1 - tx), (1, tx)):
                for dj, wy in ((0, 1 - ty), (1, ty)):
                    ii, jj = i0 + di, j0 + dj      # node index along x, y (0 = boundary)
                    if 1 <= ii <= g and 1 <= jj <= g and wx * wy != 0.0:
                        rows.append(q)
                        cols.append((jj - 1) * g + (ii - 1))
                        vals.append(wx * wy)
        self.B = np.zeros((len(pts), self.n))
        np.add.at(self.B, (np.array(rows), np.array(cols)), np.array(vals))

    def step(self, u):
        """One explicit step; u has shape (g, g, nv) indexed [iy, ix]."""
        h = self.h
        up = np.zeros((self.g + 2, self.g + 2) + u.shape[2:])
        up[1:-1, 1:-1] = u
        c = up[1:-1, 1:-1]
        dxm = (c - up[1:-1, :-2]) / h
        dxp = (up[1:-1, 2:] - c) / h
        dym = (c - up[:-2, 1:-1]) / h
        dyp = (up[2:, 1:-1] - c) / h
        vx = self.vx[..., None]
        vy = self.vy[..., None]
        adv = np.where(vx > 0, vx * dxm, vx * dxp) + np.where(vy > 0, vy * dym, vy * dyp)
        return u + self.dt * (self.kappa * _lap(u, h) - adv)

    def step_T(self, w):
        """Exact transpose of `step` (built from its stencil coefficients)."""
        h, dt, k = self.h, self.dt, self.kappa
        vx = self.vx[..., None]
        vy = self.vy[..., None]
        # coefficients of u_{iy,ix} and its neighbours in the new value at (iy,ix)
        cxm = np.where(vx > 0, vx / h, 0.0)        # weight multiplying -(c - west)
        cxp = np.where(vx > 0, 0.0, -vx / h)       # weight multiplying +(east - c) -> -vx*dxp
        cym = np.where(vy > 0, vy / h, 0.0)
        cyp = np.where(vy > 0, 0.0, -vy / h)
        d = k / (h * h)
        centre = 1.0 + dt * (-4.0 * d - cxm - cxp - cym - cyp)
        west = dt * (d + cxm)      # coefficient of u[iy, ix-1] in new u[iy, ix]
        east = dt * (d + cxp)      # coefficient of u[iy, ix+1]
        south = dt * (d + cym)     # coefficient of u[iy-1, ix]
        north = dt * (d + cyp)     # coefficient of u[iy+1, ix]
        out = centre * w
        out[:, :-1] += (west * w)[:, 1:]
        out[:, 1:] += (east * w)[:, :-1]
        out[:-1] += (south * w)[1:]
        out[1:] += (north * w)[:-1]
        return out

    def forward(self, V):
        u = V.reshape(self.g, self.g, -1).copy()
        obs = []
        for s in range(1, self.steps + 1):
            u = self.step(u)
            if s in self.obs_steps:
                obs.append(self.B @ u.reshape(self.n, -1))
        return obs

    def adjoint(self, obs):
        nv = obs[0].shape[1]
        lam = np.zeros((self.g, self.g, nv))
        for s in range(self.steps, 0, -1):
            if s in self.obs_steps:
                lam = lam + (self.B.T @ obs[self.obs_steps.index(s)]).reshape(self.g, self.g, nv)
            lam = self.step_T(lam)
        return lam.reshape(self.n, nv)

    def apply(self, V):
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        V = V.reshape(self.n, -1)
        out = self.adjoint(self.forward(V)) / (self.sigma * self.sigma)
        return out.ravel() if vec else out


class MinimalSurface:
    """Minimal-surface example of Appendix A (the surface-area objective
    minimised over the height m of a surface over the unit square, with the
    boundary heights fixed), discretised on a uniform grid.

    Reading (the paper names finite differences on a 128 x 128 grid and says
    the Hessian is exact up to discretisation): nodes (iy, ix), 0..g+1 on each
    axis, spacing h = 1/(g+1); the g x g interior heights are the unknowns
    (user index iy*g + ix), the boundary heights are data.  Each grid cell is
    cut along its anti-diagonal into a lower triangle (iy,ix),(iy,ix+1),
    (iy+1,ix) and an upper triangle (iy+1,ix+1),(iy+1,ix),(iy,ix+1); on each
    triangle the height is linear, so its gradient is the pair of one-sided
    differences along the triangle's legs, and
        J(m) = sum_T (h^2 / 2) sqrt(1 + |grad m|_T^2).
    The Hessian is exact for this J: with f(g) = sqrt(1 + |g|^2),
        d^2 f / dg^2 = ((1 + |g|^2) I - g g^T) / (1 + |g|^2)^(3/2),
    H v = sum_T (h^2 / 2) B_T^T f''(B_T m) B_T v, B_T the difference map of
    triangle T.  At a flat surface H is the 5-point Laplacian stencil
    (4 on the diagonal, -1 to each grid neighbour).
    """

    def __init__(self, cfg):
        self.g = cfg["grid"]
        self.n = self.g * self.g
        self.h = 1.0 / (self.g + 1)
        self.M = np.asarray(cfg["heights"], dtype=np.float64).reshape(self.g + 2, self.g + 2)

    def _pad(self, V):
        """Interior columns (n, nv) -> node array (g+2, g+2, nv), zero boundary."""
        nv = V.shape[1]
        P = np.zeros((self.g + 2, self.g + 2, nv))
        P[1:-1, 1:-1] = V.reshape(self.g, self.g, nv)
        return P

    def _diffs(self, P):
        """Leg differences / h on the lower and upper triangle of every cell."""
        h = self.h
        gx_lo = (P[:-1, 1:] - P[:-1, :-1]) / h
        gy_lo = (P[1:, :-1] - P[:-1, :-1]) / h
        gx_up = (P[1:, 1:] - P[1:, :-1]) / h
        gy_up = (P[1:, 1:] - P[:-1, 1:]) / h
        return gx_lo, gy_lo, gx_up, gy_up

    def _scatter(self, qx_lo, qy_lo, qx_up, qy_up):
        """sum_T (h^2/2) B_T^T q_T onto the nodes; interior part as (n, nv)."""
        h = self.h
        w = 0.5 * h * h / h
        out = np.zeros((self.g + 2, self.g + 2) + qx_lo.shape[2:])
        out[:-1, 1:] += w * qx_lo
        out[:-1, :-1] -= w * (qx_lo + qy_lo)
        out[1:, :-1] += w * qy_lo
        out[1:, 1:] += w * (qx_up + qy_up)
        out[1:, :-1] -= w * qx_up
        out[:-1, 1:] -= w * qy_up
        return out[1:-1, 1:-1].reshape(self.n, -1)

    def _with_interior(self, m):
        M = self.M.copy()
        M[1:-1, 1:-1] = np.asarray(m).reshape(self.g, self.g)
        return M

    def objective(self, m=None):
        M = self.M if m is None else self._with_interior(m)
        gx_lo, gy_lo, gx_up, gy_up = self._diffs(M)
        a = 0.5 * self.h * self.h
        return float(a * np.sum(np.sqrt(1 + gx_lo ** 2 + gy_lo ** 2))
                     + a * np.sum(np.sqrt(1 + gx_up ** 2 + gy_up ** 2)))

    def gradient(self, m=None):
        M = self.M if m is None else self._with_interior(m)
        gx_lo, gy_lo, gx_up, gy_up = self._diffs(M)
        s_lo = np.sqrt(1 + gx_lo ** 2 + gy_lo ** 2)
        s_up = np.sqrt(1 + gx_up ** 2 + gy_up ** 2)
        q = [a[..., None] for a in (gx_lo / s_lo, gy_lo / s_lo, gx_up / s_up, gy_up / s_up)]
        return self._scatter(*q)[:, 0]

    def apply(self, V):
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        V = V.reshape(self.n, -1)
        gx_lo, gy_lo, gx_up, gy_up = self._diffs(self.M)
        dx_lo, dy_lo, dx_up, dy_up = self._diffs(self._pad(V))
        q = []
        for gx, gy, dx, dy in ((gx_lo, gy_lo, dx_lo, dy_lo), (gx_up, gy_up, dx_up, dy_up)):
            s2 = 1 + gx * gx + gy * gy
            s3 = (s2 * np.sqrt(s2))[..., None]
            gx, gy = gx[..., None], gy[..., None]
            q.append(((1 + gy * gy) * dx - gx * gy * dy) / s3)
            q.append((-gx * gy * dx + (1 + gx * gx) * dy) / s3)
        out = self._scatter(q[0], q[1], q[2], q[3])
        return out.ravel() if vec else out


def tree_order(apply_user, perm):
    """Wrap a user-ordered apply so that it takes and returns tree-ordered columns."""
    def f(Om):
        Om = np.asarray(Om).reshape(len(perm), -1)
        Xu = np.empty_like(Om)
        Xu[perm] = Om
        return apply_user(Xu)[perm]
    return f


def dense_from_apply(apply_user, n, block=256):
    """H = [H e_j]_j assembled by explicit products (column blocks)."""
    H = np.empty((n, n))
    for a in range(0, n, block):
        b = min(n, a + block)
        E = np.zeros((n, b - a))
        E[np.arange(a, b), np.arange(b - a)] = 1.0
        H[:, a:b] = apply_user(E)
    return H
