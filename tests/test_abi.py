"""The C-ABI library loads and exports every symbol include/vlbm.h declares
(host-side check, no compute call, no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vlbm.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vlbm_[A-Za-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("vlbm_create", "vlbm_init", "vlbm_step", "vlbm_run_to_time", "vlbm_conserved_totals",
                 "vlbm_raw_adjoint_step"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2609_10639_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libvlbm.so not built")
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_native.EXPORTED) == declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2609_10639_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _native.lib()


def test_config_struct_matches_header_layout(tmp_path):
    """Every field of the ctypes mirror sits at the offset the C compiler gives
    it in include/vlbm.h (gcc prints offsetof for each field)."""
    import subprocess
    from paper_2609_10639_amd import _native
    fields = [f for f, _ in _native.VlbmConfig._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"vlbm.h\"\nint main(void) {\n" +
                   "".join('printf("%%zu\\n", offsetof(vlbm_config, %s));\n' % f for f in fields) +
                   'printf("%zu\\n", sizeof(vlbm_config));\nreturn 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [getattr(_native.VlbmConfig, f).offset for f in fields] + [ctypes.sizeof(_native.VlbmConfig)]
    assert got == want, list(zip(fields + ["sizeof"], got, want))

def _config(dim, nx, ny, precision):
    from paper_2609_10639_amd import _native
    c = _native.VlbmConfig()
    c.dim, c.nx, c.ny, c.dx = dim, nx, ny, 1.0 / nx
    c.eos, c.gamma, c.cfl, c.retarget_every = 0, 1.4, 0.45, 1
    c.sensor, c.beta_const, c.beta_min, c.beta_max, c.c_sensor, c.eps_theta = 2, 1.0, 0.75, 1.0, 4.0, 1e-10
    c.precision = precision
    return c


@pytest.mark.parametrize("nx,ny,precision", [(11586, 11586, 0), (16384, 8193, 0), (16384, 16385, 1),
                                             (16384, 16385, 2), (1 << 20, 1 << 12, 1)])
def test_grids_beyond_32bit_offsets_are_rejected(nx, ny, precision):
    """The D2Q4 kernels address four population planes from one buffer
    resource with 32-bit offsets; larger grids are refused by the
    configuration check, before any device call."""
    from paper_2609_10639_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libvlbm.so not built")
    lib = _native.lib()
    out = ctypes.c_void_p()
    c = _config(2, nx, ny, precision)
    assert lib.vlbm_create(ctypes.byref(c), ctypes.byref(out)) == _native.EINVAL
    assert not out.value


@pytest.mark.parametrize("nx,ny,precision,ok", [(9600, 13981, 0, True), (21301, 6301, 0, False),
                                                (19200, 13981, 1, True), (19200, 13981, 2, True),
                                                (13081, 20521, 1, False)])
def test_d2q4_size_cap_boundary(nx, ny, precision, ok):
    """The largest D2Q4 grids the 32-bit offsets allow (2^27 - 128 cells in
    FP64, 2^28 - 256 with FP32 storage: four planes of the cells rounded up to
    64 plus 1 KB fit in 4 GiB) pass the configuration check, and one cell more
    fails it (host-side check, no device call)."""
    from paper_2609_10639_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libvlbm.so not built")
    cap = (1 << 27) - 128 if precision == 0 else (1 << 28) - 256
    assert nx * ny == cap + (0 if ok else 1)
    c = _config(2, nx, ny, precision)
    assert _native.lib().vlbm_check_config(ctypes.byref(c)) == (_native.OK if ok else _native.EINVAL)


def test_status_codes_match_the_header():
    """The binding's status constants are the header's enumerators."""
    from paper_2609_10639_amd import _native
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef enum \{(.*?)\} vlbm_status;", txt, flags=re.S).group(1)
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"VLBM_(\w+)\s*=\s*(-?\d+)", body)}
    assert codes == {name: getattr(_native, name) for name in codes}
    assert codes["EDONE"] > 0 > max(v for k, v in codes.items() if k not in ("OK", "EDONE"))
    assert set(_native.STATUS_NAMES) == set(codes.values())
