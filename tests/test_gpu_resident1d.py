"""D1Q2 batches in one resident workgroup against one launch per step.

Grids of up to 2048 cells run their batches of steps in one workgroup that
keeps the populations on chip between steps (the library's default there);
VLBM_D1_RESIDENT=0 at context creation selects one launch per step, the path
larger grids take.  The two kernels run the same arithmetic in the same order,
with no fused multiply-add beyond those written out, and reduce the same
maxima, so they must agree bit for bit: populations, clock (t, c, n), step
counts, the sensor's beta, and the step and status of an inadmissible state.
Sizes cover every launch shape (2, 4 and 4 cells a lane in 256, 256 and 512
threads) at and beside its boundaries, ragged chunks included, and sizes past
the cap (one launch per step in both contexts).

Against the FP64 oracle the resident path is covered by the 1-D parity tests
at these sizes (Sod at 1000 cells, the dense-gas tube at 1024, the paper's
shock tubes at 1000 and 2000); the per-step path by the ragged-size tests
(every lane width) and by those above 2048 cells.
"""
import sys

import numpy as np
import pytest

from helpers import bzt1d_case, sod_case, tube_config
from paper_2609_10639_amd import problems as pr
from test_inflow import shu_osher_config

pytestmark = pytest.mark.gpu

PRECISIONS = ("fp64", "fp32_mixed", "fp32")
SIZES = (4, 63, 512, 513, 1000, 1024, 1025, 2048, 2049, 4095, 4096)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(monkeypatch, cfg, W0, precision):
    """(resident, one launch per step) contexts on the same input."""
    import torch
    from paper_2609_10639_amd import Solver
    assert torch.cuda.is_available()
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("VLBM_D1_RESIDENT", flag)
        s = Solver(precision=precision, **cfg)
        s.init(W0)
        out.append(s)
    monkeypatch.delenv("VLBM_D1_RESIDENT")
    return out


def _same(a, b, what):
    fa, fb = a.f(), b.f()
    assert a.clock() == b.clock(), (what, a.clock(), b.clock())
    assert np.array_equal(fa, fb), (what, np.abs(fa.astype(np.float64) - fb).max())


def _periodic(nx, sensor=1, gas=pr.IDEAL_AIR):
    W0 = pr.random_admissible_state(1, (1, nx), seed=1000 + nx, gas=gas)
    cfg = dict(dim=1, nx=nx, ny=1, dx=1.0 / nx, bc=(0, 0, 1, 1), cfl=0.5, sensor=sensor, beta_const=0.9,
               **pr.SENSOR_1D, **gas.config())
    return W0, cfg


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("nx", SIZES)
def test_periodic_steps_bitwise(monkeypatch, nx, precision):
    W0, cfg = _periodic(nx)
    _say("periodic", nx, precision)
    a, b = _pair(monkeypatch, cfg, W0, precision)
    assert a.step(150) == b.step(150) == 150
    _same(a, b, "after 150 steps")
    assert np.array_equal(a.beta(), b.beta())


def _tube(case):
    if case == "sod":
        W0, cfg, t_end = sod_case(1000)
    elif case == "bzt":
        W0, cfg, t_end = bzt1d_case(1024)
    elif case == "strong":
        W0, cfg, t_end = tube_config("strong", 2000)
    elif case == "argrow2":
        W0, cfg, t_end = tube_config("II", 3000)
    elif case == "shu_osher_pinned":
        W0, cfg, t_end = shu_osher_config(4000, "A")
    else:   # constant beta, pinned inflow, a ragged last chunk
        W0, cfg, t_end = shu_osher_config(3001, "const")
    return W0, cfg, t_end


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("case", ["sod", "bzt", "strong", "argrow2", "shu_osher_pinned", "shu_osher_beta"])
def test_tubes_to_t_end_bitwise(monkeypatch, case, precision):
    W0, cfg, t_end = _tube(case)
    _say("tube", case, cfg["nx"], precision)
    a, b = _pair(monkeypatch, cfg, W0, precision)
    na, nb = a.run_to_time(t_end), b.run_to_time(t_end)
    _say("steps", na, nb)
    assert na == nb
    assert a.clock()[0] == t_end
    _same(a, b, "at t_end")


@pytest.mark.parametrize("precision", ("fp64", "fp32"))
def test_batches_across_launches(monkeypatch, precision):
    """A batch longer than one launch of the resident kernel (4096 steps), and
    batches of every size in a row, including a landing inside a launch."""
    W0, cfg = _periodic(640)
    a, b = _pair(monkeypatch, cfg, W0, precision)
    for n in (1, 2, 9000, 3, 4096, 4097):
        assert a.step(n) == b.step(n) == n
        _same(a, b, "after a batch of %d" % n)
    t = a.clock()[0]
    t_end = t + 0.37
    na, nb = a.run_to_time(t_end), b.run_to_time(t_end)
    assert na == nb and a.clock()[0] == t_end
    _same(a, b, "after landing")
    assert a.step(5, t_end_cap=t_end) == 0   # at the cap already


def test_mixed_with_other_entry_points(monkeypatch):
    """Resident batches interleaved with the entry points that run other
    kernels on the same state: beta, totals, W, checkpoint and restore."""
    W0, cfg, _ = sod_case(1000)
    a, b = _pair(monkeypatch, cfg, W0, "fp64")
    for s in (a, b):
        s.step(100)
    assert np.array_equal(a.beta(), b.beta())
    assert np.array_equal(a.totals(), b.totals())
    ca, cb = a.save(), b.save()
    for s in (a, b):
        s.step(250)
    _same(a, b, "after 350 steps")
    a.restore(ca)
    b.restore(cb)
    _same(a, b, "restored at step 100")
    for s in (a, b):
        s.step(77)
    _same(a, b, "77 steps after the restore")
    assert np.array_equal(a.W(), b.W())


@pytest.mark.parametrize("precision", PRECISIONS)
def test_inadmissible_state_at_the_same_step(monkeypatch, precision):
    """The strong shock tube without dissipation (beta = 1, sensor off, CFL
    0.9) loses positivity at step 5 in the FP64 oracle; both paths stop at the
    same step with the same status and the same state."""
    from paper_2609_10639_amd import _native as N
    W0, dx = pr.strong_shock_tube(400)
    cfg = dict(dim=1, nx=400, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.9, sensor=0, beta_const=1.0,
               **pr.SENSOR_1D, **pr.IDEAL_AIR.config())
    a, b = _pair(monkeypatch, cfg, W0, precision)
    st = []
    for s in (a, b):
        with pytest.raises(N.VlbmError) as e:
            s.run_to_time(0.012)
        st.append(e.value.status)
    _say(precision, "status", st, "clock", a.clock(), b.clock())
    assert st[0] == st[1] and st[0] in (N.ENONHYPERBOLIC, N.ENONFINITE)
    assert 0 < a.clock()[2] < 20
    _same(a, b, "at the inadmissible state")
