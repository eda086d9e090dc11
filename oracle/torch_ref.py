"""Reference gradient of the VLBM rollout: plain PyTorch CPU FP64 ops + autograd.

TEST INFRASTRUCTURE ONLY.  The forward below is the same time step as the C
oracle with the link speed c frozen (no retarget, so no reprojection and no
landing), written with whole-grid tensor operations in the paper's order:
moments (Sec. III.A), EOS closure (Sec. II.C), flux (Eq. 10), sensor (Eqs.
28-35), relaxation towards the vector equilibrium (Eqs. 20, 22), exact
transport (Eq. 21).  Its gradient is obtained by reverse-mode automatic
differentiation, so it shares no derivation with the hand-written adjoint of
the GPU library.

Conventions at the non-smooth points of the map (shared with the library by
specification): d clip(x,0,1)/dx = 1 on the open interval (0, 1) and 0
elsewhere; the max-normaliser M_k = max_{x,alpha} |Q_alpha,k| passes its
gradient to the first maximiser in (alpha, y, x) order; d sqrt(s)/ds := 0 at
s = 0; c is a constant.
"""
import torch

DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1)]


class Frozen:
    """cfg: dict with dim, nx, ny, dx, bc (4), eos, gamma, vdw_a, vdw_b, vdw_R,
    c_fixed, sensor (0 off, 1 A, 2 B, 3 auto), beta_const, beta_min, beta_max,
    c_sensor, eps_theta.  Tensors are float64 with layout f[i, k, y, x]."""

    def __init__(self, cfg):
        self.cfg = dict(cfg)
        self.D = cfg["dim"]
        self.NK = self.D + 2
        self.Q = 2 * self.D
        self.c = float(cfg["c_fixed"])
        s = cfg.get("sensor", 3)
        self.sensor = (1 if self.D == 1 else 2) if s == 3 else s
        if self.D == 1 and self.sensor == 2:
            self.sensor = 1
        ny, nx = cfg["ny"], cfg["nx"]
        if any(b not in (0, 1) for b in cfg["bc"]):
            raise ValueError("the frozen-speed reference step covers periodic and outflow edges only")
        self.idx_x = {d: self._nb(torch.arange(nx), d, nx, cfg["bc"][0], cfg["bc"][1]) for d in (-1, 1)}
        self.idx_y = {d: self._nb(torch.arange(ny), d, ny, cfg["bc"][2], cfg["bc"][3]) for d in (-1, 1)}

    @staticmethod
    def _nb(i, d, n, lo, hi):
        j = i + d
        j = torch.where(j < 0, (j + n) if lo == 0 else torch.zeros_like(j), j)
        j = torch.where(j >= n, (j - n) if hi == 0 else torch.full_like(j, n - 1), j)
        return j

    def shift(self, a, ox, oy):
        """a evaluated at the neighbour (x + ox, y + oy), boundary rule applied."""
        if ox:
            a = a.index_select(-1, self.idx_x[ox])
        if oy:
            a = a.index_select(-2, self.idx_y[oy])
        return a

    # ---------------------------------------------------------------- EOS, flux
    def pressure(self, rho, e):
        g = self.cfg
        if g["eos"] == 0:
            return (g["gamma"] - 1.0) * rho * e
        cv = g["vdw_R"] / (g["gamma"] - 1.0)
        T = (e + g["vdw_a"] * rho) / cv
        return g["vdw_R"] * rho * T / (1.0 - g["vdw_b"] * rho) - g["vdw_a"] * rho * rho

    def flux(self, W):
        """Q[alpha][k] (Eq. 10) and the velocity components."""
        D = self.D
        rho = W[0]
        u = [W[1 + a] / rho for a in range(D)]
        e = W[D + 1] / rho - 0.5 * sum(v * v for v in u)
        P = self.pressure(rho, e)
        Q = []
        for a in range(D):
            comps = [W[1 + a]] + [W[1 + a] * u[b] + (P if a == b else 0.0) for b in range(D)] + [(W[D + 1] + P) * u[a]]
            Q.append(torch.stack(comps))
        return torch.stack(Q), u

    def equilibrium(self, W, Q):
        out = []
        for i in range(self.Q):
            cq = sum(self.c * DIRS[i][a] * Q[a] for a in range(self.D))
            out.append(W / (2.0 * self.D) + cq / (2.0 * self.c * self.c))
        return torch.stack(out)

    # ---------------------------------------------------------------- sensor
    def box(self, a):
        a = 0.25 * self.shift(a, -1, 0) + 0.5 * a + 0.25 * self.shift(a, 1, 0)
        if self.D == 2:
            a = 0.25 * self.shift(a, 0, -1) + 0.5 * a + 0.25 * self.shift(a, 0, 1)
        return a

    def beta(self, Q, u):
        g = self.cfg
        if self.sensor == 0:
            return torch.full_like(Q[0, 0], g["beta_const"])
        D, NK = self.D, self.NK
        # M_k = max over (alpha, y, x) of |Q_alpha,k|, gradient to the first maximiser
        M = []
        for k in range(NK):
            flat = Q[:, k].abs().reshape(-1)
            M.append(flat[torch.argmax(flat)])
        acc = 0.0
        for k in range(NK):
            j = 0.0
            for a in range(D):
                ox, oy = DIRS[2 * a]
                j = j + 0.5 * (self.shift(Q[a, k], ox, oy) - self.shift(Q[a, k], -ox, -oy))
            sh = torch.where(M[k] > 0, j / torch.where(M[k] > 0, M[k], torch.ones_like(M[k])), torch.zeros_like(j))
            acc = acc + sh * sh
        m = acc / NK
        pos = m > 0
        s = torch.where(pos, torch.sqrt(torch.where(pos, m, torch.ones_like(m))), torch.zeros_like(m))
        sbar = self.box(s)
        if self.sensor == 2 and D == 2:
            # dilatation and vorticity by central differences, times dt = dx/c (lattice units)
            h2, dt = 2.0 * g["dx"], g["dx"] / self.c
            dil = dt * ((self.shift(u[0], 1, 0) - self.shift(u[0], -1, 0)) / h2 + (self.shift(u[1], 0, 1) - self.shift(u[1], 0, -1)) / h2)
            vort = dt * ((self.shift(u[1], 1, 0) - self.shift(u[1], -1, 0)) / h2 - (self.shift(u[0], 0, 1) - self.shift(u[0], 0, -1)) / h2)
            theta = dil * dil / (dil * dil + vort * vort + g["eps_theta"])
            thbar = self.box(theta)
        else:
            thbar = torch.ones_like(sbar)
        x = g["c_sensor"] * sbar * thbar
        inside = (x > 0) & (x < 1)
        chi = torch.where(inside, x, torch.where(x >= 1, torch.ones_like(x), torch.zeros_like(x)).detach())
        return g["beta_max"] - (g["beta_max"] - g["beta_min"]) * chi

    # ---------------------------------------------------------------- step
    def init(self, W0):
        Q, _ = self.flux(W0)
        return self.equilibrium(W0, Q)

    def step(self, f):
        W = f.sum(0)
        Q, u = self.flux(W)
        b = self.beta(Q, u)
        fs = 2.0 * b * self.equilibrium(W, Q) + (1.0 - 2.0 * b) * f
        out = []
        for i in range(self.Q):
            ox, oy = DIRS[i]
            out.append(self.shift(fs[i], -ox, -oy))
        return torch.stack(out)

    def rollout(self, W0, nsteps):
        f = self.init(W0)
        for _ in range(nsteps):
            f = self.step(f)
        return f.sum(0)


def misfit_gradient(cfg, W0, rho_target, nsteps):
    """J = 1/2 dx^D sum (rho(T) - rho_target)^2 and dJ/dW0 (float64 numpy in/out)."""
    import numpy as np
    fr = Frozen(cfg)
    W = torch.tensor(np.asarray(W0, dtype=np.float64), requires_grad=True)
    WT = fr.rollout(W, nsteps)
    vol = cfg["dx"] ** cfg["dim"]
    J = 0.5 * vol * ((WT[0] - torch.tensor(rho_target)) ** 2).sum()
    J.backward()
    return float(J.detach()), W.grad.numpy().copy(), WT.detach().numpy()


def step_vjp(cfg, f, lam):
    """lam^n = (d step / d f)^T lam for one frozen-speed step at the state f
    (float64 numpy (Q, D+2, ny, nx) in and out)."""
    import numpy as np
    fr = Frozen(cfg)
    ft = torch.tensor(np.asarray(f, dtype=np.float64), requires_grad=True)
    out = fr.step(ft)
    out.backward(torch.tensor(np.asarray(lam, dtype=np.float64)))
    return ft.grad.numpy().copy()
