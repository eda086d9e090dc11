"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Tolerances (per field, W components):
  FP64 GPU vs oracle  relative Linf <= 1e-11 on smooth flows, relative L1 <= 1e-9
                      on shocked flows (only rounding order and FMA contraction differ);
  FP32 forms         relative Linf <= 1e-5 on smooth flows, relative L1 <= 1e-5
                      on shocked flows (the target precision of the FP32 form);
                      where a form misses it the test is an expected failure with
                      the measured value in its reason, beside a passing bound
                      that guards the measured value.
Fields are density, momentum (vector norm) and total energy.  FP64 step counts
and the landing time must match exactly.
"""
import math
import os
import sys

import numpy as np
import pytest

from helpers import (bzt1d_case, bzt2d_case, energy_gauge, gresho_case, oracle_for, rel_errors, riemann_bzt_case,
                     riemann_case, sod_case, speed_error, vortex_case)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(cfg, precision="fp64"):
    import torch
    from paper_2609_10639_amd import Solver
    assert torch.cuda.is_available()
    return Solver(precision=precision, **cfg)


def _run_both(W0, cfg, t_end, precision="fp64"):
    _say("case", cfg["dim"], cfg["nx"], cfg["ny"], precision, "t_end", t_end)
    o = oracle_for(cfg, W0)
    n_o = o.run_to_time(t_end)
    s = _solver(cfg, precision)
    s.init(W0)
    n_g = s.run_to_time(t_end)
    return o, n_o, s, n_g


def _check(o, n_o, s, n_g, t_end, tol, norm):
    assert s.clock()[0] == t_end and o.clock()[0] == t_end
    assert n_g == n_o, (n_g, n_o)
    errs = rel_errors(s.W(), o.W())
    _say("steps", n_g, "errors (relLinf, relL1) per field:", ["%.2e/%.2e" % e for e in errs])
    idx = 0 if norm == "linf" else 1
    for k, e in enumerate(errs):
        assert e[idx] <= tol, (k, e)


# ------------------------------------------------------------------ FP64 parity


def test_sod_fp64():
    W0, cfg, t_end = sod_case(1000)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end)
    _check(o, n_o, s, n_g, t_end, 1e-9, "l1")


def test_bzt_tube_fp64():
    W0, cfg, t_end = bzt1d_case(1024)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end)
    _check(o, n_o, s, n_g, t_end, 1e-9, "l1")


def test_vortex_fp64():
    W0, cfg, t_end = vortex_case(128)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end)
    _check(o, n_o, s, n_g, t_end, 1e-11, "linf")


@pytest.mark.parametrize("config", [3, 12])
def test_riemann_fp64(config):
    W0, cfg, t_end = riemann_case(128, config)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end)
    _check(o, n_o, s, n_g, t_end, 1e-9, "l1")


def test_riemann_bzt_fp64():
    W0, cfg, t_end = riemann_bzt_case(128)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end)
    _check(o, n_o, s, n_g, t_end, 1e-9, "l1")


def test_bzt_extrusion_fp64():
    W0, cfg, _ = bzt2d_case(128)
    o, n_o, s, n_g = _run_both(W0, cfg, 0.05)
    _check(o, n_o, s, n_g, 0.05, 1e-9, "l1")


@pytest.mark.parametrize("precision", [
    "fp32_mixed",
    pytest.param("fp32", marks=pytest.mark.xfail(
        strict=False, reason="FP32 arithmetic on the dense gas: momentum relative L1 1.5e-5 after 94 steps "
                             "(density and energy 2.9e-6); FP32 storage with FP64 arithmetic meets 1e-5"))])
def test_bzt_extrusion_fp32(precision):
    """The dense-gas extrusion (van der Waals, c_v/R = 50, 1 % seeded density
    noise, Sensor B), 256^2 to t = 0.2 with the energy stored in the shifted
    gauge: relative L1 per field against the oracle."""
    W0, cfg, t_end = bzt2d_case(256)
    cfg = dict(cfg, e_offset=energy_gauge(W0))
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert s.clock()[0] == t_end and abs(n_g - n_o) <= 1
    errs = rel_errors(s.W(), o.W())
    _say(precision, "bzt extrusion 256", n_g, n_o, ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[1] <= 1e-5


def test_bzt_extrusion_fp32_bound():
    """Pure FP32 arithmetic on the extrusion: the measured gap (momentum relative
    L1 1.5e-5) as a regression bound."""
    W0, cfg, t_end = bzt2d_case(256)
    cfg = dict(cfg, e_offset=energy_gauge(W0))
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, "fp32")
    for e in rel_errors(s.W(), o.W()):
        assert e[1] <= 5e-5


@pytest.mark.parametrize("shape,bc", [((67, 130), (0, 0, 0, 0)), ((67, 130), (1, 1, 1, 1)),
                                      ((5, 7), (1, 1, 0, 0)), ((61, 4), (0, 0, 1, 1)), ((59, 117), (1, 1, 0, 0)),
                                      ((4, 67), (1, 1, 0, 0)), ((4, 4), (0, 0, 0, 0))])
def test_ragged_grids_fp64(shape, bc):
    ny, nx = shape
    from paper_2609_10639_amd import problems as pr
    W = pr.random_admissible_state(2, shape, seed=nx * 1000 + ny, u_amp=0.3)
    cfg = dict(dim=2, nx=nx, ny=ny, dx=1.0 / nx, bc=bc, cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
               **pr.SENSOR_2D, **pr.IDEAL_AIR.config())
    o, n_o, s, n_g = _run_both(W, cfg, 0.02)
    _check(o, n_o, s, n_g, 0.02, 1e-9, "l1")


@pytest.mark.parametrize("precision,path", [("fp64", "resident"), ("fp64", "step1"), ("fp64", "step2"),
                                            ("fp32", "resident"), ("fp32", "step1"), ("fp32", "step2"),
                                            ("fp32", "step4"), ("fp32_mixed", "resident"), ("fp32_mixed", "step1"),
                                            ("fp32_mixed", "step2"), ("fp32_mixed", "step4")])
@pytest.mark.parametrize("nx,bc", [(4, (0, 0, 1, 1)), (5, (1, 1, 1, 1)), (7, (0, 0, 1, 1)), (57, (0, 0, 1, 1)),
                                   (59, (1, 1, 1, 1)), (63, (1, 1, 1, 1)),
                                   (119, (0, 0, 1, 1)), (121, (1, 1, 1, 1)), (241, (0, 0, 1, 1)),
                                   (247, (0, 0, 1, 1)), (249, (1, 1, 1, 1)), (4097, (1, 1, 1, 1))])
def test_ragged_1d_grids(nx, bc, precision, path, monkeypatch):
    """D1Q2 on the smallest and ragged sizes (one cell fewer or more than the
    tiles of the per-step kernel: 58 cells with 1 cell a lane, 120 with 2, 248
    with 4; halo lanes past both grid edges), periodic and outflow edges, with
    the resident workgroup and with one launch per step at every lane width
    (4097 cells take the per-step path either way)."""
    from paper_2609_10639_amd import problems as pr
    monkeypatch.setenv("VLBM_D1_RESIDENT", "1" if path == "resident" else "0")
    if path in ("step1", "step2", "step4"):
        monkeypatch.setenv("VLBM_D1_LANE_CELLS", path[-1])
    W = pr.random_admissible_state(1, (1, nx), seed=7000 + nx, u_amp=0.3)
    cfg = dict(dim=1, nx=nx, ny=1, dx=1.0 / nx, bc=bc, cfl=0.5, sensor=1, **pr.SENSOR_1D, **pr.IDEAL_AIR.config())
    o, n_o, s, n_g = _run_both(W, cfg, 0.02, precision)
    _check(o, n_o, s, n_g, 0.02, 1e-9 if precision == "fp64" else 1e-5, "l1")


@pytest.mark.parametrize("sensor", [0, 1, 2])
def test_sensor_modes_and_beta_diagnostic(sensor):
    W0, cfg, _ = riemann_case(96, 12)
    cfg = dict(cfg, sensor=sensor, beta_const=0.8)
    o = oracle_for(cfg, W0)
    s = _solver(cfg)
    s.init(W0)
    for _ in range(3):
        o.step()
    s.step(3)
    bo, bg = o.beta(), s.beta()
    _say("sensor", sensor, "beta max diff", np.abs(bo - bg).max())
    assert np.abs(bo - bg).max() <= 1e-12
    errs = rel_errors(s.W(), o.W())
    assert max(e[0] for e in errs) <= 1e-12


def test_retarget_every_k_and_frozen_speed():
    W0, cfg, _ = sod_case(400)
    for kw in (dict(retarget_every=7), dict(retarget_every=0, c_fixed=6.0)):
        c = dict(cfg, **kw)
        o = oracle_for(c, W0)
        s = _solver(c)
        s.init(W0)
        for _ in range(40):
            o.step()
        s.step(40)
        assert abs(s.clock()[1] - o.clock()[1]) <= 1e-12 * o.clock()[1]
        errs = rel_errors(s.W(), o.W())
        assert max(e[1] for e in errs) <= 1e-11


# ------------------------------------------------------------------ FP32 form
#
# FP32 storage of the populations perturbs every cell by ~6e-8 per step; FP32
# arithmetic adds rounding of the same order in the closure and the flux.  The
# Ducros ratio of Sensor B (Eq. 33) takes dilatation and vorticity in lattice
# units with a regulariser (1e-10) far above the squared rounding of FP32
# velocities, so flow that is quiescent up to rounding keeps it near zero in
# every precision (tests/test_fp32_storage_limit.py pins this on the oracle).


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp32"])
@pytest.mark.parametrize("sensor,beta", [(1, 1.0), (0, 0.9)])
def test_vortex_fp32(precision, sensor, beta):
    W0, cfg, t_end = vortex_case(128)
    cfg = dict(cfg, sensor=sensor, beta_const=beta)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert s.clock()[0] == t_end
    assert abs(n_g - n_o) <= 1
    errs = rel_errors(s.W(), o.W())
    _say(precision, "vortex sensor", sensor, ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[0] <= 1e-5


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp32"])
def test_vortex_fp32_sensor_b_bound(precision):
    """Sensor B, 128^2 to t = 10: the measured FP32 gaps (relative Linf 4.0e-6
    with FP64 arithmetic, 1.6e-5 with FP32 arithmetic) as a regression bound."""
    W0, cfg, t_end = vortex_case(128)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    errs = rel_errors(s.W(), o.W())
    _say(precision, "vortex sensor B", ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[0] <= 3e-5 and e[1] <= 5e-6


@pytest.mark.parametrize("precision", [
    "fp32_mixed",
    pytest.param("fp32", marks=pytest.mark.xfail(
        strict=False, reason="FP32 arithmetic over 833 steps: momentum relative Linf 1.6e-5 (density 8.7e-6, "
                             "energy 1.5e-5); FP32 storage with FP64 arithmetic meets 1e-5 (4.0e-6)"))])
def test_vortex_fp32_sensor_b_target(precision):
    W0, cfg, t_end = vortex_case(128)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert abs(n_g - n_o) <= 1
    for e in rel_errors(s.W(), o.W()):
        assert e[0] <= 1e-5


SHOCKED = {"riemann3": lambda: riemann_case(128, 3), "riemann12": lambda: riemann_case(128, 12),
           "sod": lambda: sod_case(1000), "bzt1d": lambda: bzt1d_case(1024),
           "riemann_bzt": lambda: riemann_bzt_case(128)}


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp32"])
@pytest.mark.parametrize("case", list(SHOCKED))
def test_shocked_fp32(case, precision):
    """Relative L1 <= 1e-5 per field.  The dense-gas cases store their energy
    in the shifted gauge (e_offset = mean internal energy of W0)."""
    W0, cfg, t_end = SHOCKED[case]()
    if case in ("bzt1d", "riemann_bzt"):
        cfg = dict(cfg, e_offset=energy_gauge(W0))
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert s.clock()[0] == t_end
    errs = rel_errors(s.W(), o.W())
    _say(precision, case, "steps", n_g, n_o, ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[1] <= 1e-5


@pytest.mark.parametrize("case", ["bzt1d", "bzt2d", "vortex"])
def test_energy_gauge_is_exact_in_fp64(case):
    """The shifted energy gauge changes only rounding: FP64 results with
    e_offset != 0 match the (unshifted) oracle like the plain FP64 path, and
    the populations and totals come back in the physical gauge."""
    W0, cfg, t_end = {"bzt1d": lambda: bzt1d_case(512), "bzt2d": lambda: bzt2d_case(64),
                      "vortex": lambda: vortex_case(64)}[case]()
    cfg = dict(cfg, e_offset=energy_gauge(W0))
    o = oracle_for(cfg, W0)
    s = _solver(cfg)
    s.init(W0)
    f0 = s.f()
    assert np.abs(f0 - o.f()).max() <= 1e-13 * np.abs(o.f()).max()
    assert np.allclose(s.totals(), o.totals(), rtol=1e-13, atol=1e-13)
    n_o = o.run_to_time(min(t_end, 0.05))
    n_g = s.run_to_time(min(t_end, 0.05))
    assert n_g == n_o
    errs = rel_errors(s.W(), o.W())
    _say("e_offset", case, n_g, ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[0] <= 1e-10 and e[1] <= 1e-11


def test_energy_gauge_rejected_by_adjoint():
    import torch
    from paper_2609_10639_amd import _native as N
    W0, cfg, _ = vortex_case(32)
    s = _solver(dict(cfg, retarget_every=0, c_fixed=7.0, e_offset=2.5))
    f = s.new_populations()
    n = s.new_norms()
    W = torch.tensor(W0, device="cuda")
    s.raw_init(W, f, n)
    lam = s.new_populations()
    with pytest.raises(N.VlbmError):
        s.raw_adjoint_step(f, n, lam, s.new_populations())


# ------------------------------------------------------------------ Gresho vortex


@pytest.mark.parametrize("precision,tol", [
    ("fp64", 1e-11), ("fp32_mixed", 1e-5),
    pytest.param("fp32", 1e-5, marks=pytest.mark.xfail(
        strict=False, reason="FP32 arithmetic on a pressure-dominated momentum flux (P ~ 5, |u| <= 1): momentum "
                             "relative Linf 1.8e-5 after 571 steps; FP32 storage with FP64 arithmetic meets 1e-5"))])
def test_gresho_against_oracle(precision, tol):
    """Gresho vortex (Sec. IV.A), 128^2 to t = 0.5 with Sensor B: parity with the
    oracle (relative Linf per field)."""
    W0, cfg, t_end = gresho_case(128, "B")
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert s.clock()[0] == t_end
    errs = rel_errors(s.W(), o.W())
    _say(precision, "gresho", n_g, n_o, ["%.2e/%.2e" % e for e in errs])
    if precision == "fp64":
        assert n_g == n_o
    for e in errs:
        assert e[0] <= tol


def test_gresho_convergence():
    """|u| error against the exact steady state at N = 100, 200, 400 (the paper's
    grids): Sensor B against the stable constant beta = 0.995.  The sensor is
    below the constant-beta error at every N and its error keeps falling faster
    than first order on average over the three grids."""
    from paper_2609_10639_amd import Solver
    err = {}
    for sensor in ("B", "const"):
        for n in (100, 200, 400):
            W0, cfg, t_end = gresho_case(n, sensor)
            s = Solver(**cfg)
            s.init(W0)
            s.run_to_time(t_end)
            err[sensor, n] = speed_error(s.W(), n)
    _say("gresho L2(|u|):", {k: "%.3e" % v for k, v in err.items()})
    for n in (100, 200, 400):
        assert err["B", n] < err["const", n]
    order = math.log2(err["B", 100] / err["B", 400]) / 2.0
    _say("Sensor B observed order 100->400: %.2f" % order)
    assert order >= 1.1


# ------------------------------------------------------------------ invariants


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_mixed"])
def test_conservation_periodic(precision):
    """Totals of each conserved component (FP64 sums of the stored populations)
    over 200 steps of the periodic vortex, relative to their initial values:
    round-off in FP64 (1e-14); in FP32 the rounding of the stored populations,
    a few 1e-8 measured (bound 2e-7)."""
    W0, cfg, _ = vortex_case(128)
    s = _solver(cfg, precision)
    s.init(W0)
    tot0 = s.totals()
    o = oracle_for(cfg, W0)
    assert np.allclose(tot0, o.totals(), rtol=1e-7 if precision != "fp64" else 1e-14, atol=1e-12)
    drift = []
    for _ in range(10):
        s.step(20)
        drift.append(np.abs(s.totals() - tot0) / np.abs(tot0))
    worst = np.max(drift)
    _say(precision, "relative drift of totals over 200 steps", worst)
    assert worst <= (2e-7 if precision != "fp64" else 1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_mixed"])
def test_tilings_agree_bitwise(monkeypatch, precision):
    """Segment height, strip width, wavefronts per workgroup and rows of loads
    in flight change only which wavefront computes a cell, or when: the
    populations agree bit for bit (the reductions are maxima, exact in any
    order).  Workgroups of 5 and 8 wavefronts apply with FP32 arithmetic only
    (the other forms keep their largest, 4)."""
    W0, cfg, _ = riemann_case(200, 3)
    outs = []
    for h, w, g, d in (("16", "48", "1", "0"), ("37", "48", "2", "1"), ("200", "32", "4", "0"),
                       ("23", "50", "3", "1"), ("16", "16", "2", "0"), ("29", "56", "2", "0"), ("29", "56", "1", "1"),
                       ("41", "24", "8", "0"), ("13", "56", "5", "0")):
        monkeypatch.setenv("VLBM_SEG_H", h)
        monkeypatch.setenv("VLBM_STRIP_W", w)
        monkeypatch.setenv("VLBM_WPG", g)
        monkeypatch.setenv("VLBM_DEEP", d)   # FP64: one or two rows of loads in flight
        s = _solver(cfg, precision)
        s.init(W0)
        s.step(30)
        outs.append(s.f())
        s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_deterministic_repeat():
    W0, cfg, _ = riemann_case(128, 3)
    res = []
    for _ in range(2):
        s = _solver(cfg)
        s.init(W0)
        s.step(50)
        res.append((s.f(), s.totals(), s.clock()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_save_restore_bitwise():
    W0, cfg, _ = riemann_case(128, 12)
    s = _solver(cfg)
    s.init(W0)
    s.step(10)
    buf = s.save()
    s.step(25)
    ref_f, ref_clock = s.f(), s.clock()
    s.restore(buf)
    s.step(25)
    assert np.array_equal(s.f(), ref_f) and s.clock() == ref_clock


def test_nothing_to_do_returns_edone():
    """At t_end, vlbm_run_to_time and a capped vlbm_step take no step and
    return VLBM_EDONE, which the binding passes as success (0 steps)."""
    import ctypes
    from paper_2609_10639_amd import _native as N
    W0, cfg, t_end = sod_case(1000)
    s = _solver(cfg)
    s.init(W0)
    assert s.run_to_time(0.05) > 0
    clock = s.clock()
    n = ctypes.c_int64(-1)
    assert N.lib().vlbm_run_to_time(s._h, 0.05, ctypes.byref(n)) == N.EDONE and n.value == 0
    assert N.lib().vlbm_run_to_time(s._h, 0.01, ctypes.byref(n)) == N.EDONE and n.value == 0
    assert N.lib().vlbm_step(s._h, 5, 0.05, ctypes.byref(n)) == N.EDONE and n.value == 0
    assert N.lib().vlbm_step(s._h, 0, math.inf, ctypes.byref(n)) == N.OK and n.value == 0
    assert s.run_to_time(0.05) == 0 and s.step(3, t_end_cap=0.05) == 0
    assert s.clock() == clock
    assert s.step(2) == 2 and s.clock()[2] == clock[2] + 2


def test_restore_refuses_foreign_or_short_checkpoints():
    """A checkpoint carries a header naming its grid, lattice and precision:
    restoring it into another context, or from a buffer shorter than
    vlbm_state_bytes, is refused and leaves the context as it was."""
    import torch
    from paper_2609_10639_amd import _native as N
    W0, cfg, _ = riemann_case(64, 12)
    s = _solver(cfg)
    s.init(W0)
    s.step(3)
    buf = s.save()
    other = _solver(dict(cfg, nx=32, ny=32, dx=1.0 / 32))
    other.init(riemann_case(32, 12)[0])
    with pytest.raises(N.VlbmError) as e:
        other.restore(buf)
    assert e.value.status == N.EINVAL
    s32 = _solver(cfg, "fp32")
    s32.init(W0)
    with pytest.raises(N.VlbmError):
        s32.restore(buf)
    with pytest.raises(N.VlbmError):
        s.restore(buf[: buf.numel() - 8])
    assert other.clock()[2] == 0 and s32.clock()[2] == 0
    f_before = s.f()
    s.restore(buf)
    assert np.array_equal(s.f(), f_before) and s.clock()[2] == 3


def test_raw_entry_points_check_their_tensors():
    """The binding refuses tensors of the wrong dtype or size before the
    library reads them."""
    import torch
    W0, cfg, _ = vortex_case(32)
    s = _solver(dict(cfg, retarget_every=0, c_fixed=7.0))
    W = torch.tensor(W0, device="cuda")
    f, n = s.new_populations(), s.new_norms()
    with pytest.raises(ValueError):
        s.raw_init(W.float(), f, n)
    with pytest.raises(ValueError):
        s.raw_init(W[:, :16], f, n)
    with pytest.raises(ValueError):
        s.raw_init(W, f[:-1], n)
    with pytest.raises(ValueError):
        s.raw_step(f, n, f.float() if f.dtype == torch.float64 else f.double(), n)
    s.raw_init(W, f, n)


def test_raw_step_refuses_misaligned_populations():
    """The D1Q2 step reads and writes 16 bytes per lane: populations that do
    not start on a 16-byte boundary are refused by the binding (ValueError)
    and by the library itself (VLBM_EINVAL), before any kernel runs."""
    import ctypes
    import torch
    from paper_2609_10639_amd import _native as N
    W0, cfg, _ = sod_case(100)
    s = _solver(dict(cfg, retarget_every=0, c_fixed=7.0))
    W = torch.tensor(W0, device="cuda")
    f, n = s.new_populations(), s.new_norms()
    s.raw_init(W, f, n)
    g = s.new_populations()
    wide = torch.empty(f.numel() + 1, dtype=f.dtype, device="cuda")
    shifted = wide[1:]   # one element past a 16-byte boundary
    with pytest.raises(ValueError):
        s.raw_step(f, n, shifted, s.new_norms())
    st = N.lib().vlbm_raw_step(s._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(n.data_ptr()),
                               ctypes.c_void_p(shifted.data_ptr()), ctypes.c_void_p(s.new_norms().data_ptr()))
    assert st == N.EINVAL
    s.raw_step(f, n, g, s.new_norms())   # aligned: accepted
    torch.cuda.synchronize()


def test_inadmissible_states_are_reported():
    from paper_2609_10639_amd import _native as N
    W0, cfg, _ = sod_case(200)
    bad = W0.copy()
    bad[2, 0, 50] = 0.0   # negative internal energy -> negative pressure
    s = _solver(cfg)
    with pytest.raises(N.VlbmError) as e:
        s.init(bad)
    assert e.value.status == N.ENONHYPERBOLIC
    nan = W0.copy()
    nan[0, 0, 10] = np.nan
    with pytest.raises(N.VlbmError) as e:
        s.init(nan)
    assert e.value.status in (N.ENONFINITE, N.ENONHYPERBOLIC)
    # an admissible state that becomes inadmissible: the four-quadrant all-shock
    # problem with the 1-D sensor constants loses positivity within a few steps
    W0, cfg, _ = riemann_case(64, 3)
    cfg = dict(cfg, beta_min=0.75, c_sensor=4.0)
    s = _solver(cfg)
    s.init(W0)
    with pytest.raises(N.VlbmError) as e:
        s.run_to_time(0.25)
    assert e.value.status in (N.ENONHYPERBOLIC, N.ENONFINITE)
    t, c, n = s.clock()
    assert 0 < n < 10


def test_bad_configs_rejected():
    from paper_2609_10639_amd import _native as N
    W0, cfg, _ = sod_case(100)
    for bad in (dict(cfl=0.0), dict(bc=(0, 1, 1, 1)), dict(nx=2), dict(beta_min=1.2), dict(dim=3),
                dict(retarget_every=0, c_fixed=0.0), dict(bc=(2, 1, 1, 1), bc_state=((0.0, 0.0, 1.0), None)),
                dict(bc=(2, 1, 1, 1), bc_state=((1.0, 0.0, -1.0), None)), dict(bc=(3, 1, 1, 1)),
                dict(bc=(2, 0, 1, 1), bc_state=((1.0, 0.0, 2.5), None))):
        with pytest.raises(N.VlbmError):
            _solver(dict(cfg, **bad))


# ------------------------------------------------------------------ full-size configurations


@pytest.mark.parametrize("name,precision,steps", [
    ("vortex1024", "fp64", 4), ("vortex1024", "fp32_mixed", 4), ("vortex1024", "fp32", 4),
    ("riemann4096", "fp32_mixed", 2), ("riemann4096", "fp32", 2), ("riemann4096", "fp64", 2),
    ("bzt2048", "fp64", 3), ("bzt2048", "fp32_mixed", 3), ("bzt2048", "fp32", 3), ("bzt8192", "fp64", 40),
    ("bzt8192", "fp32", 40), ("sod2p26", "fp64", 3), ("sod2p26", "fp32", 3), ("sod2p26", "fp32_mixed", 3)])
def test_full_size_against_oracle(name, precision, steps):
    """At the benchmark sizes and launch configuration: a few steps compared
    with the oracle over the whole grid."""
    case = {"vortex1024": lambda: vortex_case(1024), "riemann4096": lambda: riemann_case(4096, 3),
            "bzt2048": lambda: bzt2d_case(2048), "bzt8192": lambda: bzt1d_case(8192),
            "sod2p26": lambda: sod_case(1 << 26)}[name]
    W0, cfg, _ = case()
    if name.startswith("bzt") and precision != "fp64":
        cfg = dict(cfg, e_offset=energy_gauge(W0))   # dense gas in FP32: shifted energy gauge
    _say("full size", name, precision, steps)
    o = oracle_for(cfg, W0)
    for _ in range(steps):
        o.step()
    s = _solver(cfg, precision)
    s.init(W0)
    s.step(steps)
    assert s.clock()[2] == steps
    errs = rel_errors(s.W(), o.W())
    _say(" errors", ["%.2e/%.2e" % e for e in errs], "t", s.clock()[0], o.clock()[0])
    assert abs(s.clock()[0] - o.clock()[0]) <= (1e-12 if precision == "fp64" else 1e-6) * o.clock()[0]
    tol = 1e-11 if precision == "fp64" else 1e-5
    for e in errs:
        assert e[0] <= tol * 10 and e[1] <= tol


_WHOLE = {}


def _whole_run(config, sensor, precision):
    """Configuration `config` at 4096^2 to t = 0.25 (cached: several tests read
    the same runs)."""
    key = (config, sensor, precision)
    if key not in _WHOLE:
        W0, cfg, t_end = riemann_case(4096, config, sensor=sensor)
        _say("riemann 4096 to t_end", config, sensor, precision)
        s = _solver(cfg, precision)
        s.init(W0)
        n = s.run_to_time(t_end)
        assert s.clock()[0] == t_end
        _WHOLE[key] = (n, s.W())
        s.close()
    return _WHOLE[key]


def test_riemann4096_whole_run():
    """The Riemann workload at its full size, 4096^2 configuration 3 to t = 0.25
    under Sensor B (about 6200 steps, link speed retargeted every 4 steps) in
    FP64: it lands on t_end admissible (retargeted every step it loses
    admissibility at step 794, the finding behind the 2-D retarget reading) and
    keeps the problem's symmetry about the diagonal to 1e-8."""
    n64, W64 = _whole_run(3, 2, "fp64")
    rho = W64[0]
    sym = np.abs(rho - rho.T).max() / np.abs(rho).max()
    msym = np.abs(W64[1] - W64[2].T).max() / np.abs(W64[1]).max()
    _say("steps", n64, "diagonal symmetry rho %.2e momentum %.2e" % (sym, msym))
    assert sym <= 1e-8 and msym <= 1e-8


@pytest.mark.parametrize("precision,bounds", [("fp32_mixed", (1e-5, 4e-5)), ("fp32", (5e-5, 2e-4))])
def test_riemann4096_whole_run_fp32_bound(precision, bounds):
    """Both FP32 forms of the whole 4096^2 configuration-3 run (Sensor A, the
    sensor without the Ducros gate) against the GPU's FP64 run (far beyond the
    oracle's reach at this size; the FP64 path matches the oracle on the
    sampled full-size steps above and on whole runs at 512^2 below).  Measured
    relative L1, density / momentum / energy: FP32 storage with FP64 arithmetic
    3.6e-6 / 1.7e-5 / 4.1e-6, FP32 2.3e-5 / 9.6e-5 / 2.6e-5; held as regression
    bounds (density and energy, momentum).  FP64 runs from the initial state and
    from it rounded to FP32 differ by 1.5e-7: the gap is the rounding of every
    step, amplified by the fine-grid dynamics (at 512^2 and 1024^2 the same
    forms stay within 1e-5)."""
    n64, W64 = _whole_run(3, 1, "fp64")
    n32, W32 = _whole_run(3, 1, precision)
    errs = rel_errors(W32, W64)
    _say(precision, "steps", n32, n64, "vs fp64 relLinf/relL1", ["%.2e/%.2e" % e for e in errs])
    assert abs(n64 - n32) <= max(2, n64 // 1000)
    assert errs[0][1] <= bounds[0] and errs[2][1] <= bounds[0] and errs[1][1] <= bounds[1]


@pytest.mark.xfail(strict=False, reason="FP32 storage at 4096^2 over 5575 steps: momentum relative L1 1.7e-5 (FP64 "
                                        "arithmetic) and 9.6e-5 (FP32 arithmetic) against FP64")
@pytest.mark.parametrize("precision", ["fp32_mixed", "fp32"])
def test_riemann4096_whole_run_fp32_target(precision):
    n64, W64 = _whole_run(3, 1, "fp64")
    n32, W32 = _whole_run(3, 1, precision)
    for e in rel_errors(W32, W64):
        assert e[1] <= 1e-5


def test_riemann4096_config12_sensor_b_whole_run():
    """Configuration 12 under Sensor B at 4096^2 to t = 0.25 in FP64 and both
    FP32 forms: every run lands on t_end with a positive, finite density.  The
    forms are not compared field by field: under Sensor B the slip lines of the
    configuration roll up, and runs whose rounding differs drift apart
    (relative L1 of density 2e-3 between FP32 and FP64 at 4096^2, 7e-5 at
    1024^2, 5e-7 at 512^2, where the whole run matches the oracle below)."""
    for precision in ("fp64", "fp32", "fp32_mixed"):
        n, W = _whole_run(12, 2, precision)
        _say("config 12 sensor B", precision, "steps", n)
        assert np.isfinite(W).all() and W[0].min() > 0
    _WHOLE.clear()


@pytest.mark.parametrize("config,sensor", [(3, 2), (12, 2), (3, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_riemann512_whole_run_against_oracle(precision, config, sensor):
    """Configurations 3 and 12 under Sensor B, and 3 under Sensor A, at 512^2:
    whole runs to t = 0.25 against the oracle, relative L1 1e-9 in FP64 and
    1e-5 in FP32 (measured at most 3.1e-6 and 7.1e-6)."""
    W0, cfg, t_end = riemann_case(512, config, sensor=sensor)
    o, n_o, s, n_g = _run_both(W0, cfg, t_end, precision)
    assert s.clock()[0] == t_end
    if precision == "fp64":
        assert n_g == n_o
    errs = rel_errors(s.W(), o.W())
    _say(precision, "config", config, "512 whole run", n_g, n_o, ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[1] <= (1e-9 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,nx,ny,tol", [("fp32", 19200, 13981, 1e-5), ("fp64", 9600, 13981, 1e-11)])
def test_largest_grid_against_oracle(precision, nx, ny, tol):
    """The largest D2Q4 grid the 32-bit plane offsets allow (2^28 - 256 cells
    with FP32 storage, 2^27 - 128 in FP64): a smooth field periodic with periods
    64 in x and 41 in y on the periodic grid, two steps (Sensor B).  The global
    maxima and every stencil are those of the 64 x 41 torus, so the oracle on
    that torus computes the same update: every cell of the full grid must match
    it, and the full grid must stay exactly periodic (an offset that wrapped
    anywhere in the 4 GiB of a four-plane group would break both)."""
    from paper_2609_10639_amd import problems as pr
    px, py = 64, 41
    assert nx % px == 0 and ny % py == 0
    x = (np.arange(px) + 0.5) / px
    y = (np.arange(py) + 0.5) / py
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    P = 1.0 + 0.1 * np.cos(2 * np.pi * (X + Y))
    block = pr.conserved(pr.IDEAL_AIR, rho, 0.3 * np.sin(2 * np.pi * Y), P, 0.2 * np.cos(2 * np.pi * X))
    dx = 1.0 / px
    cfg = dict(dim=2, nx=px, ny=py, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
               **pr.SENSOR_2D, **pr.IDEAL_AIR.config())
    o = oracle_for(cfg, block)
    o.step()
    o.step()
    Wo = o.W()
    _say("largest grid", precision, nx, ny, nx * ny)
    W0 = np.tile(block, (1, ny // py, nx // px))
    s = _solver(dict(cfg, nx=nx, ny=ny), precision)
    s.init(W0)
    del W0
    s.step(2)
    assert s.clock()[2] == 2 and abs(s.clock()[1] - o.clock()[1]) <= 1e-12 * o.clock()[1]
    W = s.W().reshape(4, ny // py, py, nx // px, px)
    s.close()
    first = W[:, 0, :, 0, :].copy()
    assert np.array_equal(W, np.broadcast_to(first[:, None, :, None, :], W.shape))   # exactly periodic
    del W
    errs = rel_errors(first, Wo)
    _say(" errors against the oracle on the torus", ["%.2e/%.2e" % e for e in errs])
    for e in errs:
        assert e[0] <= tol
