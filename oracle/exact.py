"""Exact solutions used to pin the oracle (test infrastructure only).

* Exact Riemann solution of the 1-D ideal-gas Euler equations (the Sod tube of
  the shock-tube configuration), by the classical pressure-function method:
  the star pressure p* solves f_L(p) + f_R(p) + u_R - u_L = 0, where f_K is the
  velocity jump across a shock (Rankine-Hugoniot) or a rarefaction (isentropic
  Riemann invariant) connecting state K to pressure p.
* Error norms (domain-mean L1, L2, Linf, relative L1 and Linf).
"""
import math

import numpy as np
from scipy.optimize import brentq


class IdealRiemann:
    def __init__(self, left, right, gamma=1.4):
        self.g = gamma
        self.L = tuple(map(float, left))
        self.R = tuple(map(float, right))
        self.aL = math.sqrt(gamma * self.L[2] / self.L[0])
        self.aR = math.sqrt(gamma * self.R[2] / self.R[0])
        self.p_star, self.u_star = self._solve()

    def _f(self, p, K, a):
        g = self.g
        rho, _, pK = K
        if p > pK:  # shock: Rankine-Hugoniot mass/momentum jump
            A = 2.0 / ((g + 1.0) * rho)
            B = (g - 1.0) / (g + 1.0) * pK
            return (p - pK) * math.sqrt(A / (p + B))
        # rarefaction: constant Riemann invariant u +- 2a/(g-1) along the isentrope
        return 2.0 * a / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def _solve(self):
        du = self.R[1] - self.L[1]
        F = lambda p: self._f(p, self.L, self.aL) + self._f(p, self.R, self.aR) + du
        hi = max(self.L[2], self.R[2])
        while F(hi) < 0:
            hi *= 2.0
        p = brentq(F, 1e-14 * hi, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        u = 0.5 * (self.L[1] + self.R[1]) + 0.5 * (self._f(p, self.R, self.aR) - self._f(p, self.L, self.aL))
        return p, u

    def star_densities(self):
        g, ps = self.g, self.p_star
        out = []
        for K in (self.L, self.R):
            rho, _, p = K
            if ps > p:
                r = ps / p
                k = (g - 1.0) / (g + 1.0)
                out.append(rho * (r + k) / (k * r + 1.0))
            else:
                out.append(rho * (ps / p) ** (1.0 / g))
        return tuple(out)

    def wave_speeds(self):
        """(left head, left tail or left shock, contact, right tail, right head)."""
        g, ps, us = self.g, self.p_star, self.u_star
        rsL, rsR = self.star_densities()
        rho, u, p = self.L
        if ps > p:
            sL = u - self.aL * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            hL = tL = sL
        else:
            hL = u - self.aL
            tL = us - math.sqrt(g * ps / rsL)
        rho, u, p = self.R
        if ps > p:
            sR = u + self.aR * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            hR = tR = sR
        else:
            hR = u + self.aR
            tR = us + math.sqrt(g * ps / rsR)
        return hL, tL, us, tR, hR

    def sample(self, xi):
        """Primitive state (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
        g, ps, us = self.g, self.p_star, self.u_star
        xi = np.asarray(xi, dtype=np.float64)
        rho = np.empty_like(xi)
        u = np.empty_like(xi)
        p = np.empty_like(xi)
        rsL, rsR = self.star_densities()
        hL, tL, _, tR, hR = self.wave_speeds()
        for side in (0, 1):
            K = self.L if side == 0 else self.R
            aK = self.aL if side == 0 else self.aR
            rs = rsL if side == 0 else rsR
            sgn = -1.0 if side == 0 else 1.0
            head, tail = (hL, tL) if side == 0 else (hR, tR)
            m = xi < us if side == 0 else xi >= us
            x = xi[m]
            # outer (unperturbed) region, fan, star region
            outer = (x < head) if side == 0 else (x > head)
            star = (x >= tail) if side == 0 else (x <= tail)
            fan = ~outer & ~star
            r = np.empty_like(x)
            uu = np.empty_like(x)
            pp = np.empty_like(x)
            r[outer], uu[outer], pp[outer] = K
            r[star], uu[star], pp[star] = rs, us, ps
            if np.any(fan):
                # inside a centred rarefaction: the characteristic dx/dt = u -+ a
                # passes through the origin, with the Riemann invariant of state K
                a = 2.0 / (g + 1.0) * (aK - sgn * (g - 1.0) / 2.0 * (K[1] - x[fan]))
                uu[fan] = 2.0 / (g + 1.0) * (-sgn * aK + (g - 1.0) / 2.0 * K[1] + x[fan])
                r[fan] = K[0] * (a / aK) ** (2.0 / (g - 1.0))
                pp[fan] = K[2] * (a / aK) ** (2.0 * g / (g - 1.0))
            rho[m], u[m], p[m] = r, uu, pp
        return rho, u, p


def norms(num, ref):
    """Domain-mean L1, RMS L2, Linf, relative L1 and relative Linf."""
    d = np.abs(np.asarray(num) - np.asarray(ref))
    aref = np.abs(np.asarray(ref))
    return dict(L1=d.mean(), L2=math.sqrt((d * d).mean()), Linf=d.max(),
                relL1=d.sum() / max(aref.sum(), 1e-300), relLinf=d.max() / max(aref.max(), 1e-300))


def primitives(W, gamma=1.4):
    """Ideal-gas (rho, u[, v], P) from W; used only to compare with exact solutions."""
    D = W.shape[0] - 2
    rho = W[0]
    vel = [W[1 + a] / rho for a in range(D)]
    ke = sum(0.5 * v * v for v in vel)
    P = (gamma - 1.0) * (W[D + 1] - rho * ke)
    return (rho, *vel, P)


def gresho_speed(n):
    """|u| of the steady Gresho vortex (Sec. IV.A) at the centres of an n x n
    grid on [0, 1]^2: 5r for r < 0.2, 2 - 5r for 0.2 <= r < 0.4, 0 beyond."""
    import numpy as np
    c = (np.arange(n) + 0.5) / n - 0.5
    r = np.sqrt(c[None, :] ** 2 + c[:, None] ** 2)
    return np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
