"""ctypes declarations of libvlbm.so (include/vlbm.h).  Argument marshalling only.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any entry point.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlbm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONHYPERBOLIC, ENONFINITE, EDONE = 0, -1, -2, -3, -4, -5, 1
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONHYPERBOLIC", -5: "ENONFINITE",
                1: "EDONE"}
BC_PERIODIC, BC_OUTFLOW, BC_PINNED = 0, 1, 2
EOS_IDEAL, EOS_VDW = 0, 1
SENSOR_OFF, SENSOR_A, SENSOR_B, SENSOR_AUTO = 0, 1, 2, 3
FP64, FP32, FP32_MIXED = 0, 1, 2
NORMS_LEN = 256   # doubles in a norms array (VLBM_NORMS_LEN)


class VlbmConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("dx", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4),
        ("bc_state", (ctypes.c_double * 4) * 2),
        ("eos", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("vdw_a", ctypes.c_double),
        ("vdw_b", ctypes.c_double),
        ("vdw_R", ctypes.c_double),
        ("e_offset", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("retarget_every", ctypes.c_int32),
        ("c_fixed", ctypes.c_double),
        ("sensor", ctypes.c_int32),
        ("beta_const", ctypes.c_double),
        ("beta_min", ctypes.c_double),
        ("beta_max", ctypes.c_double),
        ("c_sensor", ctypes.c_double),
        ("eps_theta", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class VlbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None

# (name, restype, argtypes)
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = [
    ("vlbm_check_config", ctypes.c_int, [ctypes.POINTER(VlbmConfig)]),
    ("vlbm_create", ctypes.c_int, [ctypes.POINTER(VlbmConfig), ctypes.POINTER(ctypes.c_void_p)]),
    ("vlbm_destroy", None, [_P]),
    ("vlbm_init", ctypes.c_int, [_P, _P, ctypes.c_int32]),
    ("vlbm_step", ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    ("vlbm_run_to_time", ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    ("vlbm_conserved_totals", ctypes.c_int, [_P, _D]),
    ("vlbm_get_W", ctypes.c_int, [_P, _P, ctypes.c_int32]),
    ("vlbm_get_beta", ctypes.c_int, [_P, _P, ctypes.c_int32]),
    ("vlbm_get_f", ctypes.c_int, [_P, _P, ctypes.c_int32]),
    ("vlbm_get_clock", ctypes.c_int, [_P, _D, _D, ctypes.POINTER(ctypes.c_int64)]),
    ("vlbm_state_bytes", ctypes.c_size_t, [_P]),
    ("vlbm_save", ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    ("vlbm_restore", ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    ("vlbm_plane_elems", ctypes.c_int64, [_P]),
    ("vlbm_population_bytes", ctypes.c_size_t, [_P]),
    ("vlbm_raw_init", ctypes.c_int, [_P, _P, _P, _P]),
    ("vlbm_raw_step", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("vlbm_raw_adjoint_step", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("vlbm_raw_adjoint_step_static", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("vlbm_raw_init_adjoint", ctypes.c_int, [_P, _P, _P, _P]),
    ("vlbm_raw_moments", ctypes.c_int, [_P, _P, _P]),
    ("vlbm_raw_moments_adjoint", ctypes.c_int, [_P, _P, _P]),
    ("vlbm_last_error", ctypes.c_char_p, [_P]),
    ("vlbm_copy_probe", ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, ctypes.c_int32]),
    ("vlbm_copy_probe_read_bytes", ctypes.c_size_t, [ctypes.c_size_t]),
    ("vlbm_probe_march", ctypes.c_int, [_P, ctypes.c_int32]),
]
EXPORTED = [name for name, _, _ in _SIGS]


def lib():
    """Load libvlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvlbm.so is not built (run __graft_entry__.build() or "
                               "python paper_2609_10639_amd/build.py); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, handle=None):
    """Raise VlbmError for an error status; OK and EDONE (nothing to do) pass."""
    if status not in (OK, EDONE):
        msg = lib().vlbm_last_error(handle).decode() if handle else ""
        raise VlbmError(status, msg)


def copy_probe(src, dst, nbytes, stream, mode=0):
    """vlbm_copy_probe: device-to-device copy of nbytes (mode 0), or a read-only
    stream over src folded into per-workgroup XOR words in dst (mode 1), through
    the library's bandwidth probe kernels (a measurement aid), stream-ordered."""
    check(lib().vlbm_copy_probe(src, dst, nbytes, stream, mode))
