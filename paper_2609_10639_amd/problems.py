"""Seeded synthetic inputs for the VLBM hot path.

This module only builds initial conditions: primitive states of the paper's
benchmark families, converted to the conserved vector W = (rho, rho u, rho E)
(Sec. II.A, Eqs. 1-2) through the caloric relation e(rho, P) of the chosen EOS,
plus a counter-based random number generator.  The shock-vortex problem also
needs its exact stationary-shock states and an EOS-generic vortex; those are
solved here from thermodynamic relations written out from the van der Waals
model itself (isentrope, sound speed as -v^2 dP/dv along it, enthalpy).  It holds none of the method's
arithmetic (no flux, equilibrium, sensor or time step) and both the CPU oracle
and the GPU library consume the arrays it returns unchanged.

Arrays are float64, shape (D+2, ny, nx) with ny == 1 in 1-D, cell centres at
x_j = (j + 1/2) dx.
"""
import math

import numpy as np

# --------------------------------------------------------------- RNG

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, idx):
    """Counter-based SplitMix64 (Steele, Lea & Flood 2014): the (idx+1)-th
    output of the generator seeded with `seed`, for an array of counters."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed, n):
    """n uniforms in [0, 1): top 53 bits of SplitMix64 times 2^-53."""
    z = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def gaussian(seed, n):
    """n standard normals by Box-Muller on the uniform pairs (2m, 2m+1)."""
    m = (n + 1) // 2
    u = uniform(seed, 2 * m)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log1p(-u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    out = np.empty(2 * m)
    out[0::2] = z[:m]
    out[1::2] = z[m:]
    return out[:n]


# --------------------------------------------------------------- EOS parameters

IDEAL, VDW = 0, 1


class Gas:
    """EOS parameters.  Ideal gas: gamma.  van der Waals: a, b, R and gamma with
    c_v = R/(gamma - 1) (Sec. II.C)."""

    def __init__(self, eos=IDEAL, gamma=1.4, a=0.0, b=0.0, R=1.0):
        self.eos, self.gamma, self.a, self.b, self.R = eos, gamma, a, b, R

    @property
    def cv(self):
        return self.R / (self.gamma - 1.0)

    def internal_energy(self, rho, P):
        """Specific internal energy e(rho, P): ideal P/((gamma-1) rho);
        vdW T = (P + a rho^2)(1 - b rho)/(R rho), e = c_v T - a rho (Eqs. 16-17)."""
        rho = np.asarray(rho, dtype=np.float64)
        P = np.asarray(P, dtype=np.float64)
        if self.eos == IDEAL:
            return P / ((self.gamma - 1.0) * rho)
        T = (P + self.a * rho * rho) * (1.0 - self.b * rho) / (self.R * rho)
        return self.cv * T - self.a * rho

    def config(self):
        return dict(eos=self.eos, gamma=self.gamma, vdw_a=self.a, vdw_b=self.b, vdw_R=self.R)


IDEAL_AIR = Gas(IDEAL, 1.4)
IDEAL_MONO = Gas(IDEAL, 5.0 / 3.0)
# reduced van der Waals units rho_c = P_c = 1 (a = 3, b = 1/3, R = 1), c_v/R = 50
VDW_REDUCED_CV50 = Gas(VDW, 1.0 + 1.0 / 50.0, 3.0, 1.0 / 3.0, 1.0)
# the BZT van der Waals gas of Sec. IV.F and IV.H: a = 1, b = 0.3, R = 1, c_v/R = 50
BZT_GAS = Gas(VDW, 1.02, 1.0, 0.3, 1.0)


def conserved(gas, rho, u, P, v=None):
    """(rho, u[, v], P) -> W = (rho, rho u[, rho v], rho E), E = e + |u|^2/2."""
    rho = np.asarray(rho, dtype=np.float64)
    e = gas.internal_energy(rho, P)
    ke = 0.5 * u * u + (0.5 * v * v if v is not None else 0.0)
    comps = [rho, rho * u] + ([rho * v] if v is not None else []) + [rho * (e + ke)]
    return np.stack([np.broadcast_to(c, rho.shape) for c in comps]).astype(np.float64)


def centres(n, lo, hi):
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx, dx


# --------------------------------------------------------------- sensor settings

# (beta_min, beta_max, C_sensor) of Sec. III.D.  1-D: the values the paper states
# for its strong shock tube.  2-D: beta_min = 0.7, the largest constant beta
# that keeps the all-shock four-quadrant problem admissible, and C = 16, the
# smallest of 4, 8, 16 with which the sensor keeps it admissible.
SENSOR_1D = dict(beta_min=0.75, beta_max=1.0, c_sensor=4.0)
SENSOR_2D = dict(beta_min=0.7, beta_max=1.0, c_sensor=16.0)

# Regulariser of the Ducros ratio (Eq. 33), a dimensionless number: dilatation
# and vorticity enter in lattice units (dt times their central differences).
# 1e-10 is a velocity difference of 1e-5 link speeds across one cell, squared:
# far below any compression the gate has to see, far above the squared
# rounding of FP32 populations (about 1e-14), so that flow that is quiescent up
# to rounding keeps theta near 0 in every precision.
EPS_THETA = 1e-10

# Link-speed retargeting of the D2Q4 workloads (Sec. III.E allows a subset of
# the time steps; the paper states every step for its 1-D runs only): every 4
# steps, and at once whenever s_max exceeds c.  Retargeting every step makes
# the link speed follow s_max step by step; where beta is near 1 the lattice's
# grid-scale modes are barely damped, they enter s_max, and the step-to-step
# change of c and its reprojection feed them back (the all-shock four-quadrant
# problem under Sensor B, and the dense-gas extrusion with its cell-scale noise,
# lose admissibility from 800^2 and 1024^2 up; a frozen c, or a retarget every
# 2, 4 or 10 steps, keeps both admissible to their end times at every grid).
RETARGET_2D = 4

# --------------------------------------------------------------- 1-D problems


def shock_tube(n, left, right, gas=IDEAL_AIR, x0=0.5, lo=0.0, hi=1.0):
    """Riemann problem on [lo, hi]: (rho, u, P) = left for x < x0, right after."""
    x, dx = centres(n, lo, hi)
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    P = np.where(L, left[2], right[2])
    W = conserved(gas, rho, u, P)
    return W.reshape(3, 1, n), dx


def sod(n=1000):
    """Sod tube: (1, 0, 1) | (0.125, 0, 0.1), ideal gamma = 1.4, [0, 1]."""
    return shock_tube(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))


def strong_shock_tube(n=2000):
    """Strong shock tube (Sec. IV.C): (1, 0, 1000) | (1, 0, 0.01), ideal
    gamma = 1.4, [0, 1], discontinuity at x = 1/2."""
    return shock_tube(n, (1.0, 0.0, 1000.0), (1.0, 0.0, 0.01))


# Argrow van der Waals shock tubes (Sec. IV.D): reduced units a = 3, b = 1/3,
# R = 1; per case R/c_v, left and right (rho, u, P) and the end time.
ARGROW_CASES = {
    "I": dict(R_over_cv=0.0125, left=(0.879, 0.0, 1.09), right=(0.562, 0.0, 0.885), t_end=0.45),
    "II": dict(R_over_cv=0.329, left=(1.01, 0.0, 1.6077), right=(0.594, 0.0, 0.8957), t_end=0.20),
    "III": dict(R_over_cv=0.0125, left=(1.818, 0.0, 3.00), right=(0.275, 0.0, 0.575), t_end=0.15),
}


def argrow_gas(case):
    """van der Waals gas of an Argrow case: gamma = 1 + R/c_v."""
    return Gas(VDW, 1.0 + ARGROW_CASES[case]["R_over_cv"], 3.0, 1.0 / 3.0, 1.0)


def argrow_tube(n, case):
    c = ARGROW_CASES[case]
    return shock_tube(n, c["left"], c["right"], gas=argrow_gas(case))


def shu_osher(n=5000):
    """Shu-Osher problem (Sec. IV.B) on [-5, 5]: (3.857143, 2.629369, 10.33333)
    for x < -4, else (1 + 0.2 sin 5x, 0, 1); ideal gamma = 1.4."""
    x, dx = centres(n, -5.0, 5.0)
    L = x < -4.0
    rho = np.where(L, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(L, 2.629369, 0.0)
    P = np.where(L, 10.33333, 1.0)
    return conserved(IDEAL_AIR, rho, u, P).reshape(3, 1, n), dx


# BZT tube states in reduced vdW units (c_v/R = 50): the paper's south-east and
# north-east quadrant states of its BZT Riemann problem (Eq. 49, a = 1, b = 0.3),
# converted by rho/rho_c, P/P_c, u/sqrt(P_c/rho_c) with rho_c = 1/(3b),
# P_c = a/(27 b^2), the normal velocity taken along the tube.
BZT_LEFT = (0.9, -0.25875, 1.005923)
BZT_RIGHT = (0.585, 0.0, 0.893341)


def bzt_tube(n=8192):
    return shock_tube(n, BZT_LEFT, BZT_RIGHT, gas=VDW_REDUCED_CV50)


# --------------------------------------------------------------- 2-D problems


def isentropic_vortex_primitives(X, Y, t=0.0, L=10.0, strength=5.0, gamma=1.4,
                                 centre=(5.0, 5.0), background=(1.0, 1.0)):
    """Yee/Shu isentropic vortex advected by a uniform background flow.

    Azimuthal speed u_phi = strength/(2 pi) r exp((1 - r^2)/2) (core radius 1),
    closed by dP/dr = rho u_phi^2/r along the isentrope P = rho^gamma with
    rho = P = 1 far away (Sec. IV.H): T = P/rho = 1 - (gamma-1) strength^2/(8 gamma pi^2)
    exp(1 - r^2).  The centre at time t is centre + background*t, taken to the
    nearest periodic image on [0, L)^2."""
    cx = (centre[0] + background[0] * t) % L
    cy = (centre[1] + background[1] * t) % L
    dxp = (X - cx + 0.5 * L) % L - 0.5 * L
    dyp = (Y - cy + 0.5 * L) % L - 0.5 * L
    r2 = dxp * dxp + dyp * dyp
    amp = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = background[0] - amp * dyp
    v = background[1] + amp * dxp
    T = 1.0 - (gamma - 1.0) * strength ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    P = rho * T
    return rho, u, v, P


def vortex(n, L=10.0, strength=5.0, t=0.0):
    """Periodic [0, L]^2 isentropic vortex, centre (5, 5), background (1, 1)."""
    x, dx = centres(n, 0.0, L)
    X, Y = np.meshgrid(x, x)
    rho, u, v, P = isentropic_vortex_primitives(X, Y, t=t, L=L, strength=strength)
    return conserved(IDEAL_AIR, rho, u, P, v), dx


def vortex_in_stream(nx, ny, dx, speed=2.0, centre=None, strength=5.0):
    """Isentropic vortex (the Yee/Shu profile above, rho = P = 1 far away) in a
    uniform stream (speed, 0) on [0, nx dx] x [0, ny dx], periodic images in y
    only.  Returns W and the free-stream state (1, speed, 0, 1) as conserved
    variables: the state to hold at an upstream pinned edge."""
    Lx, Ly = nx * dx, ny * dx
    cx, cy = centre if centre is not None else (0.5 * Lx, 0.5 * Ly)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    dxp = X - cx
    dyp = (Y - cy + 0.5 * Ly) % Ly - 0.5 * Ly
    r2 = dxp * dxp + dyp * dyp
    g = IDEAL_AIR.gamma
    amp = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - (g - 1.0) * strength ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (g - 1.0))
    W = conserved(IDEAL_AIR, rho, speed - amp * dyp, rho * T, amp * dxp)
    W_inf = conserved(IDEAL_AIR, np.ones(1), np.full(1, speed), np.ones(1), np.zeros(1))[:, 0]
    return W, W_inf


# --------------------------------------------------------------- shock-vortex


def temperature(gas, rho, P):
    """T(rho, P): ideal P/(R rho); van der Waals (P + a rho^2)(1 - b rho)/(R rho)."""
    if gas.eos == IDEAL:
        return P / (gas.R * rho)
    return (P + gas.a * rho * rho) * (1.0 - gas.b * rho) / (gas.R * rho)


def sound_speed2(gas, rho, P):
    """c_s^2 = -v^2 (dP/dv) at constant entropy, v = 1/rho.  With constant c_v
    the isentropes are T (v - b)^(R/c_v) = const, so for van der Waals
    c_s^2 = gamma R T/(1 - b rho)^2 - 2 a rho, and gamma P/rho for the ideal gas."""
    if gas.eos == IDEAL:
        return gas.gamma * P / rho
    T = temperature(gas, rho, P)
    return gas.gamma * gas.R * T / (1.0 - gas.b * rho) ** 2 - 2.0 * gas.a * rho


def enthalpy(gas, rho, P):
    return gas.internal_energy(rho, P) + P / rho


def isentrope_pressure(gas, rho, rho0, P0):
    """P(rho) on the isentrope through (rho0, P0): T = T0 [(v0 - b)/(v - b)]^(R/c_v)."""
    T0 = temperature(gas, rho0, P0)
    b = gas.b if gas.eos == VDW else 0.0
    T = T0 * ((1.0 / rho0 - b) / (1.0 / rho - b)) ** (gas.R / gas.cv)
    if gas.eos == IDEAL:
        return gas.R * rho * T
    return gas.R * rho * T / (1.0 - gas.b * rho) - gas.a * rho * rho


def stationary_shock(gas, rho1, P1, mach):
    """Downstream state (rho2, u2, P2) of a stationary normal shock with
    upstream (rho1, u1 = mach c_s1, P1) (Sec. IV.H): the root rho2 > rho1 of the
    mass, momentum and stagnation-enthalpy jump conditions
        rho1 u1 = rho2 u2,  rho1 u1^2 + P1 = rho2 u2^2 + P2,  h1 + u1^2/2 = h2 + u2^2/2,
    bracketed on a fine scan of rho2 and refined by bisection.  Returns
    (u1, (rho2, u2, P2))."""
    u1 = mach * math.sqrt(sound_speed2(gas, rho1, P1))
    m = rho1 * u1
    mom = rho1 * u1 * u1 + P1
    H = enthalpy(gas, rho1, P1) + 0.5 * u1 * u1

    def resid(r2):
        u2 = m / r2
        return enthalpy(gas, r2, mom - m * u2) + 0.5 * u2 * u2 - H

    hi = (1.0 - 1e-9) / gas.b if (gas.eos == VDW and gas.b > 0) else 20.0 * rho1
    xs = np.linspace(rho1 * (1.0 + 1e-6), hi, 20001)
    fs = np.array([resid(x) for x in xs])
    k = np.nonzero(fs[:-1] * fs[1:] < 0)[0]
    if len(k) == 0:
        raise ValueError("no compressive shock root")
    lo, up = xs[k[0]], xs[k[0] + 1]
    for _ in range(200):
        mid = 0.5 * (lo + up)
        if resid(lo) * resid(mid) <= 0:
            up = mid
        else:
            lo = mid
    r2 = 0.5 * (lo + up)
    return u1, (r2, m / r2, mom - m * m / r2)


def vortex_profile(gas, rho_inf, P_inf, strength=2.0, core=1.0, r_max=12.0, h=1e-3):
    """EOS-generic isentropic vortex (Sec. IV.H): azimuthal speed
    u_phi = strength/(2 pi core) r exp((1 - r^2/core^2)/2) with the density from
    d rho/dr = rho u_phi^2/(r c_s^2) along the isentrope through the far field
    (rho_inf, P_inf), integrated inward from r_max by Heun's RK2.  Returns the
    ascending radii and rho(r)."""
    def uphi2_over_r(r):
        return (strength / (2.0 * math.pi * core)) ** 2 * r * math.exp(1.0 - r * r / (core * core))

    def rhs(r, rho):
        return rho * uphi2_over_r(r) / sound_speed2(gas, rho, isentrope_pressure(gas, rho, rho_inf, P_inf))

    n = int(round(r_max / h))
    rs = np.linspace(0.0, r_max, n + 1)
    rho = np.empty(n + 1)
    rho[n] = rho_inf
    for i in range(n, 0, -1):
        r, dr = rs[i], rs[i - 1] - rs[i]
        k1 = rhs(r, rho[i])
        k2 = rhs(r + dr, rho[i] + dr * k1)
        rho[i - 1] = rho[i] + 0.5 * dr * (k1 + k2)
    return rs, rho


# (rho1, P1) ambient states of Sec. IV.H and their runs: ideal gas and the BZT
# van der Waals gas
SHOCK_VORTEX = {
    "ideal": dict(gas=IDEAL_AIR, rho1=1.0, P1=1.0, nx=800, ny=300, t_end=7.0),
    "bzt": dict(gas=BZT_GAS, rho1=0.70, P1=0.3787, nx=1200, ny=450, t_end=15.0),
}


def shock_vortex(case, nx=None, ny=None, mach=1.2, Lx=16.0, Ly=6.0, xs=6.0, centre=(2.0, 3.0), strength=2.0):
    """Stationary normal shock at x = xs in its rest frame on [0, Lx] x [0, Ly]
    with the upstream state for x < xs, the exact downstream state beyond, and
    an isentropic vortex (core radius 1) centred at `centre` superposed on the
    upstream cells only (Sec. IV.H).  Returns W, dx and the upstream conserved
    state (the state of the pinned inflow edge)."""
    c = SHOCK_VORTEX[case]
    gas = c["gas"]
    nx = nx or c["nx"]
    ny = ny or c["ny"]
    dx = Lx / nx
    if abs(Ly / ny - dx) > 1e-12 * dx:
        raise ValueError("square cells need ny/nx = Ly/Lx")
    u1, (r2, u2, P2) = stationary_shock(gas, c["rho1"], c["P1"], mach)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    ox, oy = X - centre[0], Y - centre[1]
    r = np.hypot(ox, oy)
    rs, prof = vortex_profile(gas, c["rho1"], c["P1"], strength)
    rho_v = np.interp(r, rs, prof)
    uphi = strength / (2.0 * math.pi) * r * np.exp(0.5 * (1.0 - r * r))
    safe = np.maximum(r, 1e-300)
    up = X < xs
    rho = np.where(up, rho_v, r2)
    u = np.where(up, u1 - uphi * oy / safe, u2)
    v = np.where(up, uphi * ox / safe, 0.0)
    P = np.where(up, isentrope_pressure(gas, rho_v, c["rho1"], c["P1"]), P2)
    W = conserved(gas, rho, u, P, v)
    W_in = conserved(gas, np.full(1, c["rho1"]), np.full(1, u1), np.full(1, c["P1"]), np.zeros(1))[:, 0]
    return W, dx, W_in


def vortex_perturbed(n, amplitude=1e-3, seed=42, L=10.0, strength=5.0):
    """Vortex initial state plus amplitude * N(0, 1) on every component of W,
    independent per cell and component (seeded SplitMix64 + Box-Muller)."""
    W, dx = vortex(n, L, strength)
    xi = gaussian(seed, W.size).reshape(W.shape)
    return W + amplitude * xi, dx


def gresho(n, P0=5.0):
    """Gresho vortex on the periodic [0, 1]^2 (Sec. IV.A): rho = 1, gamma = 5/3,
    azimuthal speed 5r (r < 0.2), 2 - 5r (0.2 <= r < 0.4), 0 beyond, about the
    centre (1/2, 1/2), with the pressure that balances it; a steady solution."""
    x, dx = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x)
    ox, oy = X - 0.5, Y - 0.5
    r = np.hypot(ox, oy)
    uphi = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
    rs = np.maximum(r, 1e-300)
    P = np.where(r < 0.2, P0 + 12.5 * r * r,
                 np.where(r < 0.4, P0 + 12.5 * r * r + 4.0 * (1.0 - 5.0 * r - math.log(0.2) + np.log(rs)),
                          P0 - 2.0 + 4.0 * math.log(2.0)))
    # (u, v) = u_phi (-sin phi, cos phi) with sin phi = oy/r, cos phi = ox/r
    u = np.where(r > 0, -uphi * oy / rs, 0.0)
    v = np.where(r > 0, uphi * ox / rs, 0.0)
    return conserved(IDEAL_MONO, np.ones_like(X), u, P, v), dx


# Four-quadrant states (rho, u, v, P) of the paper's 2-D Riemann problems:
# configurations 12 and 3 (ideal gas, Sec. IV.E) and the BZT problem (Sec. IV.F,
# Eq. 49), with each one's gas and end time.
RIEMANN_CONFIGS = {
    12: dict(NE=(0.5313, 0.0, 0.0, 0.4), NW=(1.0, 0.7276, 0.0, 1.0),
             SW=(0.8, 0.0, 0.0, 1.0), SE=(1.0, 0.0, 0.7276, 1.0)),
    3: dict(NE=(1.5, 0.0, 0.0, 1.5), NW=(0.5323, 1.206, 0.0, 0.3),
            SW=(0.138, 1.206, 1.206, 0.029), SE=(0.5323, 0.0, 1.206, 0.3)),
    "bzt": dict(NE=(0.65000, 0.0, 0.0, 0.36763), NW=(1.00051, 0.15803, 0.0, 0.41396),
                SW=(0.75000, 0.0, 0.0, 0.41396), SE=(1.00000, 0.0, -0.15747, 0.41396)),
}
RIEMANN_GAS = {12: IDEAL_AIR, 3: IDEAL_AIR, "bzt": BZT_GAS}
RIEMANN_T_END = {12: 0.25, 3: 0.3, "bzt": 0.35}


def riemann2d(n, config=3):
    """Four-quadrant problem on [0, 1]^2, discontinuities along x = y = 1/2.
    With an odd n the centre row and column (x or y exactly 1/2) belong to the
    east and north quadrants, so every cell is assigned."""
    x, dx = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x)
    st = RIEMANN_CONFIGS[config]
    rho = np.zeros_like(X)
    u = np.zeros_like(X)
    v = np.zeros_like(X)
    P = np.zeros_like(X)
    east, north = X >= 0.5, Y >= 0.5
    for q, mask in (("NE", east & north), ("NW", ~east & north), ("SW", ~east & ~north), ("SE", east & ~north)):
        rho[mask], u[mask], v[mask], P[mask] = st[q]
    return conserved(RIEMANN_GAS[config], rho, u, P, v), dx


def bzt_extrusion(n=2048, noise=0.01, seed=1234):
    """BZT tube extruded along y with rho *= 1 + noise (2U - 1), U seeded uniform,
    velocity and pressure held (internal energy recomputed)."""
    x, dx = centres(n, 0.0, 1.0)
    X = np.broadcast_to(x[None, :], (n, n))
    L = X < 0.5
    rho = np.where(L, BZT_LEFT[0], BZT_RIGHT[0])
    u = np.where(L, BZT_LEFT[1], BZT_RIGHT[1])
    P = np.where(L, BZT_LEFT[2], BZT_RIGHT[2])
    U = uniform(seed, n * n).reshape(n, n)
    rho = rho * (1.0 + noise * (2.0 * U - 1.0))
    return conserved(VDW_REDUCED_CV50, rho, u, P, np.zeros_like(rho)), dx


def random_admissible_state(D, shape, seed, gas=IDEAL_AIR, rho_range=(0.5, 1.5),
                            u_amp=0.5, P_range=(0.5, 1.5)):
    """Smooth-free random admissible states for identity checks."""
    n = int(np.prod(shape))
    U = uniform(seed, (D + 2) * n).reshape(D + 2, *shape)
    rho = rho_range[0] + (rho_range[1] - rho_range[0]) * U[0]
    vel = [u_amp * (2 * U[1 + a] - 1) for a in range(D)]
    P = P_range[0] + (P_range[1] - P_range[0]) * U[D + 1]
    if D == 1:
        return conserved(gas, rho, vel[0], P)
    return conserved(gas, rho, vel[0], P, vel[1])
