"""Shared test helpers: run the oracle and the GPU library on the same inputs."""
import numpy as np

from oracle import core, muscl
from paper_2609_10639_amd import problems as pr

# workloads: (builder, config) pairs with the paper's boundary and sensor choices
IDEAL = pr.IDEAL_AIR.config()
VDW = pr.VDW_REDUCED_CV50.config()


def sod_case(n=1000):
    W0, dx = pr.sod(n)
    return W0, dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.5, sensor=1, **pr.SENSOR_1D, **IDEAL), 0.2


def bzt1d_case(n=1024):
    W0, dx = pr.bzt_tube(n)
    return W0, dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.5, sensor=1, **pr.SENSOR_1D, **VDW), 0.2


def vortex_case(n=128):
    W0, dx = pr.vortex(n)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                    **pr.SENSOR_2D, **IDEAL), 10.0


def riemann_case(n=128, config=3, sensor=2):
    """Four-quadrant problem to t = 0.25, outflow, Sensor B (or the sensor given)."""
    W0, dx = pr.riemann2d(n, config)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 1, 1), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=sensor,
                    **pr.SENSOR_2D, **IDEAL), 0.25


def riemann_bzt_case(n=128):
    """BZT four-quadrant problem (Sec. IV.F, Eq. 49) to t = 0.35, outflow, Sensor B."""
    W0, dx = pr.riemann2d(n, "bzt")
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 1, 1), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                    **pr.SENSOR_2D, **pr.BZT_GAS.config()), pr.RIEMANN_T_END["bzt"]


def bzt2d_case(n=256):
    W0, dx = pr.bzt_extrusion(n)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                    **pr.SENSOR_2D, **VDW), 0.2


def energy_gauge(W0):
    """Mean specific internal energy of W0: the e_offset that centres the stored
    energy component of FP32 populations."""
    D = W0.shape[0] - 2
    rho = W0[0]
    ke = 0.5 * sum(W0[1 + a] ** 2 for a in range(D)) / rho
    return float(np.mean((W0[D + 1] - ke) / rho))


def gresho_case(n=100, sensor="B"):
    """Gresho vortex to t = 0.5 (Sec. IV.A): Sensor B with beta_min equal to the
    stable constant beta 0.995 (the paper's rule for beta_min), or that
    constant beta alone."""
    W0, dx = pr.gresho(n)
    cfg = dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D,
               **pr.IDEAL_MONO.config())
    if sensor == "B":
        cfg.update(sensor=2, beta_min=0.995, beta_max=1.0, c_sensor=16.0)
    else:
        cfg.update(sensor=0, beta_const=0.995)
    return W0, cfg, 0.5


def speed_error(W, n):
    """L2 (root mean square) error of |u| against the steady Gresho solution."""
    from oracle.exact import gresho_speed
    sp = np.hypot(W[1] / W[0], W[2] / W[0])
    return float(np.sqrt(np.mean((sp - gresho_speed(n)) ** 2)))


def oracle_for(cfg, W0):
    kw = {k: v for k, v in cfg.items() if k not in ("precision", "e_offset")}
    o = core.Oracle(**kw)
    o.init(W0)
    return o


def rel_errors(a, b):
    """Relative Linf and relative L1 of a against reference b for each physical
    field: density, momentum (as a vector: |rho u - rho u_ref| over |rho u_ref|,
    so a component that happens to be near zero is not divided by itself) and
    total energy."""
    D = b.shape[0] - 2
    fields = [(a[0:1], b[0:1]), (a[1:1 + D], b[1:1 + D]), (a[D + 1:D + 2], b[D + 1:D + 2])]
    out = []
    for x, y in fields:
        d = np.sqrt(((x - y) ** 2).sum(axis=0))
        ref = np.sqrt((y ** 2).sum(axis=0))
        out.append((d.max() / max(ref.max(), 1e-300), d.sum() / max(ref.sum(), 1e-300)))
    return out


# ------------------------------------------- the paper's 1-D shock tubes


def tube_primitives(W, gas):
    """(rho, u, P) of a 1-D state under the gas's EOS, written out here."""
    rho = W[0, 0]
    u = W[1, 0] / rho
    e = W[2, 0] / rho - 0.5 * u * u
    if gas.eos == pr.IDEAL:
        P = (gas.gamma - 1.0) * rho * e
    else:
        T = (e + gas.a * rho) / gas.cv
        P = gas.R * rho * T / (1.0 - gas.b * rho) - gas.a * rho * rho
    return rho, u, P


def _tube(case):
    if case == "strong":
        return pr.strong_shock_tube, pr.IDEAL_AIR, 0.012
    return (lambda n: pr.argrow_tube(n, case)), pr.argrow_gas(case), pr.ARGROW_CASES[case]["t_end"]


def tube_config(case, n):
    """D1Q2 configuration of the paper's shock tubes: outflow ends, CFL 0.8,
    Sensor A with (0.75, 1, 4) (Sec. IV.C, reused for Sec. IV.D)."""
    build, gas, t_end = _tube(case)
    W0, dx = build(n)
    cfg = dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.8, sensor=1,
               **pr.SENSOR_1D, **gas.config())
    return W0, cfg, t_end


def reference_primitives(case, n, n_ref):
    """MUSCL reference at n_ref cells, cell-averaged onto n cells."""
    build, gas, t_end = _tube(case)
    m = n_ref // n
    W0, dx = build(n_ref)
    W, _ = muscl.run(W0, 1, n_ref, 1, dx, (1, 1, 1, 1), t_end, **gas.config())
    return tube_primitives(W.reshape(3, 1, n, m).mean(axis=3), gas)


def l1_errors(case, W, n, n_ref):
    _, gas, _ = _tube(case)
    ref = reference_primitives(case, n, n_ref)
    return dict(zip(("rho", "u", "P"), (float(np.mean(np.abs(a - b))) for a, b in zip(tube_primitives(W, gas), ref))))
