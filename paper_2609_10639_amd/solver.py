"""Python face of the C ABI: a Solver owning one vlbm_ctx.

Marshalling only: arrays go in and out as numpy (host) or torch (device)
buffers, the stream is torch's current HIP stream, and every step of the
method runs in the library's HIP kernels.
"""
import ctypes
import math

import numpy as np

from . import _native as N


def _torch():
    import torch
    return torch


class Solver:
    """VLBM solver on the current GPU.

    Keyword arguments follow `vlbm_config` (include/vlbm.h): dim, nx, ny, dx,
    bc (4-tuple; 0 periodic, 1 outflow, 2 pinned), bc_state (pair of conserved
    states held at pinned x-low / x-high edges, None where unused), eos, gamma, vdw_a, vdw_b, vdw_R, e_offset, cfl, retarget_every,
    c_fixed, sensor, beta_const, beta_min, beta_max, c_sensor, eps_theta,
    precision ("fp64" | "fp32" | "fp32_mixed": FP32 populations with FP64 arithmetic).
    """

    DEFAULTS = dict(dim=1, nx=100, ny=1, dx=0.01, bc=(1, 1, 1, 1), eos=0, gamma=1.4, vdw_a=0.0, vdw_b=0.0,
                    vdw_R=1.0, e_offset=0.0, cfl=0.5, retarget_every=1, c_fixed=0.0, sensor=3, beta_const=1.0, beta_min=0.75,
                    beta_max=1.0, c_sensor=4.0, eps_theta=1e-10, precision="fp64")

    def __init__(self, stream=None, **kw):
        torch = _torch()
        d = dict(self.DEFAULTS)
        d.update(kw)
        self.params = d
        cfg = N.VlbmConfig()
        for k, v in d.items():
            if k == "bc":
                for j in range(4):
                    cfg.bc[j] = int(v[j])
            elif k == "bc_state":
                for side in range(2):
                    for j, w in enumerate(v[side] if v[side] is not None else ()):
                        cfg.bc_state[side][j] = float(w)
            elif k == "precision":
                cfg.precision = {"fp64": N.FP64, "fp32": N.FP32, "fp32_mixed": N.FP32_MIXED}.get(v, v)
            else:
                setattr(cfg, k, v)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        cfg.stream = ctypes.c_void_p(stream.cuda_stream)
        self.cfg = cfg
        self.D = d["dim"]
        self.NK = self.D + 2
        self.Q = 2 * self.D
        self.shape = (d["ny"], d["nx"])
        self.fp32 = cfg.precision in (N.FP32, N.FP32_MIXED)
        h = ctypes.c_void_p()
        st = N.lib().vlbm_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != N.OK:
            raise N.VlbmError(st, "vlbm_create rejected the configuration")
        self._h = h

    # ------------------------------------------------------------ lifecycle
    def close(self):
        side = getattr(self, "_rollout_side", None)   # second context of an overlapped adjoint rollout
        if side is not None:
            self._rollout_side = None
            side[1].close()
        if getattr(self, "_h", None) is not None:
            N.lib().vlbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        N.check(st, self._h)

    # ------------------------------------------------------------ state
    def init(self, W0):
        """W0: numpy float64 (D+2, ny, nx) on the host, or a torch float64 device tensor."""
        torch = _torch()
        if isinstance(W0, torch.Tensor):
            W0 = W0.to(dtype=torch.float64).contiguous()
            assert W0.is_cuda and W0.numel() == self.NK * self.shape[0] * self.shape[1]
            self._keep = W0
            self._chk(N.lib().vlbm_init(self._h, ctypes.c_void_p(W0.data_ptr()), 1))
        else:
            W0 = np.ascontiguousarray(W0, dtype=np.float64)
            assert W0.size == self.NK * self.shape[0] * self.shape[1]
            self._chk(N.lib().vlbm_init(self._h, W0.ctypes.data_as(ctypes.c_void_p), 0))

    def step(self, nsteps=1, t_end_cap=math.inf):
        n = ctypes.c_int64(0)
        self._chk(N.lib().vlbm_step(self._h, int(nsteps), float(t_end_cap), ctypes.byref(n)))
        return n.value

    def run_to_time(self, t_end):
        n = ctypes.c_int64(0)
        self._chk(N.lib().vlbm_run_to_time(self._h, float(t_end), ctypes.byref(n)))
        return n.value

    def clock(self):
        t, c, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        self._chk(N.lib().vlbm_get_clock(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(n)))
        return t.value, c.value, n.value

    def totals(self):
        out = np.empty(self.NK)
        self._chk(N.lib().vlbm_conserved_totals(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def W(self, device=False):
        if device:
            torch = _torch()
            out = torch.empty((self.NK,) + self.shape, dtype=torch.float64, device="cuda")
            self._chk(N.lib().vlbm_get_W(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty((self.NK,) + self.shape)
        self._chk(N.lib().vlbm_get_W(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def beta(self):
        out = np.empty(self.shape)
        self._chk(N.lib().vlbm_get_beta(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def f(self):
        out = np.empty((self.Q, self.NK) + self.shape, dtype=np.float32 if self.fp32 else np.float64)
        self._chk(N.lib().vlbm_get_f(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def state_bytes(self):
        return N.lib().vlbm_state_bytes(self._h)

    def save(self):
        """Checkpoint into a new uint8 device tensor."""
        torch = _torch()
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device="cuda")
        self._chk(N.lib().vlbm_save(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))
        return buf

    def restore(self, buf):
        """Resume from a checkpoint of save(): a contiguous uint8 device tensor
        (the library refuses one taken on another grid, lattice or precision)."""
        torch = _torch()
        if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous() and buf.dtype == torch.uint8):
            raise ValueError("restore needs the contiguous uint8 device tensor that save() returned")
        self._chk(N.lib().vlbm_restore(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))

    # ------------------------------------------------------------ raw (frozen link speed)
    def plane_elems(self):
        return N.lib().vlbm_plane_elems(self._h)

    def new_populations(self):
        torch = _torch()
        dt = torch.float32 if self.fp32 else torch.float64
        return torch.empty((self.Q * self.NK, self.plane_elems()), dtype=dt, device="cuda")

    def new_norms(self):
        torch = _torch()
        return torch.zeros(N.NORMS_LEN, dtype=torch.float64, device="cuda")

    def probe_march(self, nlaunch=1):
        """Measurement aid: the step's access pattern without its arithmetic
        (vlbm_probe_march), stream-ordered; the state is left as it was."""
        self._chk(N.lib().vlbm_probe_march(self._h, int(nlaunch)))

    # The raw entry points read and write whole device arrays through plain
    # pointers: every tensor is checked for device, layout, dtype and size here,
    # so that a wrong one raises instead of being read past its end.
    def _pop(self, t):
        torch = _torch()
        return _ptr(t, torch.float32 if self.fp32 else torch.float64, self.Q * self.NK * self.plane_elems(),
                    "populations")

    def _nrm(self, t):
        return _ptr(t, _torch().float64, N.NORMS_LEN, "norms")

    def _fld(self, t):
        return _ptr(t, _torch().float64, self.NK * self.shape[0] * self.shape[1], "W")

    def raw_init(self, W0, f0, norms0):
        self._chk(N.lib().vlbm_raw_init(self._h, self._fld(W0), self._pop(f0), self._nrm(norms0)))

    def raw_step(self, f_in, norms_in, f_out, norms_out):
        self._chk(N.lib().vlbm_raw_step(self._h, self._pop(f_in), self._nrm(norms_in), self._pop(f_out),
                                        self._nrm(norms_out)))

    def raw_adjoint_step(self, f_n, norms_n, lam_np1, lam_n):
        self._chk(N.lib().vlbm_raw_adjoint_step(self._h, self._pop(f_n), self._nrm(norms_n), self._pop(lam_np1),
                                                self._pop(lam_n)))

    def raw_adjoint_step_static(self, f_n, norms_n, lam_np1, lam_n):
        """raw_adjoint_step with the library's static scratch: allocates nothing."""
        self._chk(N.lib().vlbm_raw_adjoint_step_static(self._h, self._pop(f_n), self._nrm(norms_n),
                                                       self._pop(lam_np1), self._pop(lam_n)))

    def raw_init_adjoint(self, W0, lam0, W0bar):
        self._chk(N.lib().vlbm_raw_init_adjoint(self._h, self._fld(W0), self._pop(lam0), self._fld(W0bar)))

    def raw_moments(self, f, W):
        self._chk(N.lib().vlbm_raw_moments(self._h, self._pop(f), self._fld(W)))

    def raw_moments_adjoint(self, Wbar, lam):
        self._chk(N.lib().vlbm_raw_moments_adjoint(self._h, self._fld(Wbar), self._pop(lam)))


def _ptr(t, dtype, numel, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s: a contiguous device tensor is needed" % what)
    if t.dtype != dtype or t.numel() != numel:
        raise ValueError("%s: expected %d elements of %s, got %d of %s" % (what, numel, dtype, t.numel(), t.dtype))
    if t.data_ptr() % 16:
        raise ValueError("%s: the tensor must start on a 16-byte boundary" % what)
    return ctypes.c_void_p(t.data_ptr())
