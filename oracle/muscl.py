"""ctypes wrapper of the reference finite-volume solver (muscl.c).

TEST INFRASTRUCTURE ONLY: an independent numerical method (MUSCL reconstruction
of the primitive variables with the minmod limiter, Rusanov flux, RK2) that
supplies reference solutions where no closed form exists, as the paper does
for its shock-tube and Riemann benchmarks (Sec. IV.B-IV.F).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "muscl.c")
_LIB = os.path.join(_HERE, "libmuscl_ref.so")


class MsConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double),
                ("bc", ctypes.c_int * 4), ("bc_state", (ctypes.c_double * 4) * 2), ("eos", ctypes.c_int), ("gamma", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("cfl", ctypes.c_double)]


def build(force=False):
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _get():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.ms_run.argtypes = [ctypes.POINTER(MsConfig), ctypes.POINTER(ctypes.c_double), ctypes.c_double]
        L.ms_run.restype = ctypes.c_long
        L.ms_state.argtypes = [ctypes.POINTER(MsConfig), ctypes.c_double, ctypes.c_double,
                               ctypes.POINTER(ctypes.c_double)]
        L.ms_state.restype = None
        _lib = L
    return _lib


def _config(dim=1, nx=1, ny=1, dx=1.0, bc=(1, 1, 1, 1), cfl=0.4, eos=0, gamma=1.4, vdw_a=0.0, vdw_b=0.0,
            vdw_R=1.0, bc_state=(None, None)):
    c = MsConfig()
    c.dim, c.nx, c.ny, c.dx = dim, nx, ny, dx
    for i in range(4):
        c.bc[i] = int(bc[i])
    for side in range(2):
        for j, w in enumerate(bc_state[side] if bc_state[side] is not None else ()):
            c.bc_state[side][j] = float(w)
    c.eos, c.gamma, c.a, c.b, c.R, c.cfl = eos, gamma, vdw_a, vdw_b, vdw_R, cfl
    return c


def state(rho, P, eos=0, gamma=1.4, vdw_a=0.0, vdw_b=0.0, vdw_R=1.0, **_):
    """(e, P, c_s^2) of this solver's EOS at density rho and pressure P."""
    out = (ctypes.c_double * 3)()
    _get().ms_state(ctypes.byref(_config(eos=eos, gamma=gamma, vdw_a=vdw_a, vdw_b=vdw_b, vdw_R=vdw_R)),
                    float(rho), float(P), out)
    return tuple(out)


def run(W0, dim, nx, ny, dx, bc, t_end, cfl=0.4, eos=0, gamma=1.4, vdw_a=0.0, vdw_b=0.0, vdw_R=1.0,
        bc_state=(None, None), **_):
    """Advance W0 ((dim+2, ny, nx) FP64) to t_end with periodic (0), outflow (1)
    or pinned (2, x edges, state bc_state[side]) boundaries bc = (x-low, x-high,
    y-low, y-high); returns (W, steps)."""
    c = _config(dim, nx, ny, dx, bc, cfl, eos, gamma, vdw_a, vdw_b, vdw_R, bc_state)
    W = np.ascontiguousarray(np.array(W0, dtype=np.float64))
    steps = _get().ms_run(ctypes.byref(c), W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t_end))
    if steps < 0:
        raise RuntimeError("reference solver: inadmissible state")
    return W, steps
