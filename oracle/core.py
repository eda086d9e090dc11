"""ctypes wrapper of the plain FP64 CPU oracle (vlbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vlbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_vlbm.so")

PERIODIC, OUTFLOW, PINNED = 0, 1, 2
IDEAL, VDW = 0, 1
SENSOR_OFF, SENSOR_A, SENSOR_B, SENSOR_AUTO = 0, 1, 2, 3
OK, LANDED = 0, 1


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nx", ctypes.c_long),
        ("ny", ctypes.c_long),
        ("dx", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("bc_state", (ctypes.c_double * 4) * 2),
        ("eos", ctypes.c_int),
        ("gamma", ctypes.c_double),
        ("vdw_a", ctypes.c_double),
        ("vdw_b", ctypes.c_double),
        ("vdw_R", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("retarget_every", ctypes.c_int),
        ("c_fixed", ctypes.c_double),
        ("sensor", ctypes.c_int),
        ("beta_const", ctypes.c_double),
        ("beta_min", ctypes.c_double),
        ("beta_max", ctypes.c_double),
        ("c_sensor", ctypes.c_double),
        ("eps_theta", ctypes.c_double),
    ]


def build(force=False):
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.orc_create.argtypes = [P(OrcConfig), P(ctypes.c_void_p)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_threads.restype = ctypes.c_int
        L.orc_init.argtypes = [ctypes.c_void_p, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_run_to_time.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_long, P(ctypes.c_long)]
        L.orc_beta.argtypes = [ctypes.c_void_p, dp]
        L.orc_get_W.argtypes = [ctypes.c_void_p, dp]
        L.orc_get_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_get_clock.argtypes = [ctypes.c_void_p, dp, dp, P(ctypes.c_long)]
        L.orc_set_clock.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_long]
        L.orc_set_clock.restype = None
        L.orc_get_clock.restype = None
        L.orc_reproject.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_reproject.restype = None
        L.orc_totals.argtypes = [ctypes.c_void_p, dp]
        L.orc_eos.argtypes = [P(OrcConfig), ctypes.c_double, ctypes.c_double, dp]
        L.orc_eos.restype = None
        L.orc_gamma_fundamental.argtypes = [P(OrcConfig), ctypes.c_double, ctypes.c_double]
        L.orc_gamma_fundamental.restype = ctypes.c_double
        L.orc_equilibrium.argtypes = [P(OrcConfig), ctypes.c_double, dp, dp]
        L.orc_equilibrium.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_config(**kw):
    """Build an OrcConfig from keyword arguments (same names as the fields)."""
    d = dict(dim=1, nx=100, ny=1, dx=0.01, bc=(OUTFLOW,) * 4, eos=IDEAL, gamma=1.4, vdw_a=0.0,
             vdw_b=0.0, vdw_R=1.0, cfl=0.5, retarget_every=1, c_fixed=0.0, sensor=SENSOR_AUTO,
             beta_const=1.0, beta_min=0.75, beta_max=1.0, c_sensor=4.0, eps_theta=1e-10)
    d.update(kw)
    cfg = OrcConfig()
    for k, v in d.items():
        if k == "bc":
            for j in range(4):
                cfg.bc[j] = int(v[j])
        elif k == "bc_state":
            # ((W_b at x-low), (W_b at x-high)): conserved states of pinned edges
            for side in range(2):
                for j, w in enumerate(v[side] if v[side] is not None else ()):
                    cfg.bc_state[side][j] = float(w)
        else:
            setattr(cfg, k, v)
    return cfg


class Oracle:
    """FP64 CPU reference solver.  W arrays are (D+2, ny, nx) float64."""

    def __init__(self, **kw):
        self.cfg = make_config(**kw)
        self.D = self.cfg.dim
        self.NK = self.D + 2
        self.Q = 2 * self.D
        self.shape = (self.cfg.ny, self.cfg.nx)
        h = ctypes.c_void_p()
        st = lib().orc_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if st != 0:
            raise ValueError("orc_create failed: %d" % st)
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    def init(self, W0):
        W0 = np.ascontiguousarray(W0, dtype=np.float64).reshape(self.NK, *self.shape)
        st = lib().orc_init(self._h, _dp(W0))
        if st != 0:
            raise RuntimeError("orc_init failed: %d" % st)

    def step(self, t_end=np.inf):
        return lib().orc_step(self._h, float(t_end))

    def run_to_time(self, t_end, max_steps=10**9):
        n = ctypes.c_long(0)
        st = lib().orc_run_to_time(self._h, float(t_end), int(max_steps), ctypes.byref(n))
        if st < 0:
            raise RuntimeError("oracle step failed: %d" % st)
        return n.value

    def W(self):
        out = np.empty((self.NK,) + self.shape)
        lib().orc_get_W(self._h, _dp(out))
        return out

    def f(self):
        out = np.empty((self.Q, self.NK) + self.shape)
        lib().orc_get_f(self._h, _dp(out))
        return out

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.NK, *self.shape)
        lib().orc_set_f(self._h, _dp(f))

    def beta(self):
        out = np.empty(self.shape)
        st = lib().orc_beta(self._h, _dp(out))
        if st != 0:
            raise RuntimeError("orc_beta failed: %d" % st)
        return out

    def clock(self):
        t, c, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_long()
        lib().orc_get_clock(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(n))
        return t.value, c.value, n.value

    def set_clock(self, t, c, n):
        lib().orc_set_clock(self._h, float(t), float(c), int(n))

    def reproject(self, c_new):
        lib().orc_reproject(self._h, float(c_new))

    def totals(self):
        out = np.empty(self.NK)
        lib().orc_totals(self._h, _dp(out))
        return out


def threads():
    """OpenMP threads the oracle's loops run on."""
    return int(lib().orc_threads())


def eos(cfg, rho, e):
    out = np.empty(4)
    lib().orc_eos(ctypes.byref(cfg), float(rho), float(e), _dp(out))
    return dict(P=out[0], cs2=out[1], P_rho=out[2], P_e=out[3])


def gamma_fundamental(cfg, rho, e):
    return lib().orc_gamma_fundamental(ctypes.byref(cfg), float(rho), float(e))


def equilibrium(cfg, c, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    D = cfg.dim
    out = np.empty((2 * D, D + 2))
    lib().orc_equilibrium(ctypes.byref(cfg), float(c), _dp(W), _dp(out))
    return out
