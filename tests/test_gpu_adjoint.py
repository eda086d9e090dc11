"""GPU adjoint: gradients of a terminal density misfit with respect to the
initial state, from the library's hand-written adjoint (through the C ABI and
the autograd wrapper), against the reference gradient (PyTorch CPU FP64
autograd of the frozen-speed forward, pinned to finite differences of the C
oracle) and against central finite differences of the GPU forward.

Tolerances: FP64 adjoint vs reference gradient, relative L2 <= 1e-9 (only
rounding order differs); FP64 adjoint vs central differences at full size,
1e-4 per direction; FP32 forms, relative L2 <= 1e-3 against the reference on
small grids and against the FP64 adjoint at full size (Sensor A; 3e-3 for pure
FP32 arithmetic over 625 steps).  With Sensor B at full size (the adjoint
workload) FP32 storage with FP64 arithmetic meets 1e-3; FP32 arithmetic misses
it (expected failure with the measured value, beside a passing bound).

Inputs with piecewise-constant states (Sod, Riemann, BZT) carry a seeded
perturbation: exact ties of the max-normalisers M_k between plateau cells make
the map non-differentiable there, and two correct implementations then pick
different subgradients.
"""
import sys

import numpy as np
import pytest
import torch

from oracle.torch_ref import misfit_gradient
from paper_2609_10639_amd import problems as pr

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _vortex_cfg(n, c=None):
    W0, dx = pr.vortex_perturbed(n, amplitude=1e-3, seed=42)
    cfg = dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), retarget_every=0,
               c_fixed=c if c else 2.93 / 0.45, sensor=2, **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, beta_const=1.0,
               **pr.IDEAL_AIR.config())
    return W0, cfg


def _gpu_gradient(cfg, W0, rho_t, nsteps, precision, checkpoint_every=None, overlap=True):
    from paper_2609_10639_amd import Solver
    from paper_2609_10639_amd.adjoint import rollout
    s = Solver(precision=precision, **cfg)
    W = torch.tensor(W0, device="cuda", requires_grad=True)
    WT = rollout(W, s, nsteps, checkpoint_every, overlap)
    vol = cfg["dx"] ** cfg["dim"]
    J = 0.5 * vol * ((WT[0] - torch.tensor(rho_t, device="cuda")) ** 2).sum()
    J.backward()
    return float(J), W.grad.cpu().numpy(), WT.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _noisy(W, amp=1e-3, seed=9):
    """Seeded perturbation of every component: keeps the maximisers of the
    normalisers M_k unique (ties between cells are non-differentiable points)."""
    return W + amp * np.abs(W).max(axis=(1, 2), keepdims=True) * pr.gaussian(seed, W.size).reshape(W.shape)


CASES = {
    "vortex_periodic_B": lambda: _vortex_cfg(48),
    "riemann12_outflow_B": lambda: (_noisy(pr.riemann2d(40, 12)[0]),
                                    dict(dim=2, nx=40, ny=40, dx=1 / 40, bc=(1, 1, 1, 1), retarget_every=0, c_fixed=4.5,
                                         sensor=2, **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, beta_const=1.0,
                                         **pr.IDEAL_AIR.config())),
    "bzt_mixed_B": lambda: (_noisy(pr.bzt_extrusion(32)[0]),
                            dict(dim=2, nx=32, ny=32, dx=1 / 32, bc=(1, 1, 0, 0), retarget_every=0, c_fixed=1.9,
                                 sensor=2, **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, beta_const=1.0,
                                 **pr.VDW_REDUCED_CV50.config())),
    "vortex_A": lambda: (_vortex_cfg(40)[0], dict(_vortex_cfg(40)[1], sensor=1)),
    "vortex_const_beta": lambda: (_vortex_cfg(40)[0], dict(_vortex_cfg(40)[1], sensor=0, beta_const=0.9)),
    "sod_1d": lambda: (_noisy(pr.sod(128)[0]), dict(dim=1, nx=128, ny=1, dx=1 / 128, bc=(1, 1, 1, 1), retarget_every=0,
                                             c_fixed=5.0, sensor=1, **pr.SENSOR_1D, eps_theta=pr.EPS_THETA,
                                             beta_const=1.0, **pr.IDEAL_AIR.config())),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_adjoint_matches_reference_gradient(name):
    W0, cfg = CASES[name]()
    steps = 10
    rng_t = W0[0] + 0.01 * pr.gaussian(5, W0[0].size).reshape(W0[0].shape)
    _say("adjoint case", name, cfg["nx"], cfg["ny"], steps)
    J_ref, g_ref, WT_ref = misfit_gradient(cfg, W0, rng_t, steps)
    J, g, WT = _gpu_gradient(cfg, W0, rng_t, steps, "fp64", checkpoint_every=3)
    _say(" forward rel diff", _rel(WT, WT_ref), "gradient rel L2", _rel(g, g_ref))
    assert _rel(WT, WT_ref) <= 1e-12
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
    assert _rel(g, g_ref) <= 1e-9


@pytest.mark.parametrize("precision", ["fp32", "fp32_mixed"])
def test_fp32_adjoint_against_reference(precision):
    W0, cfg = _vortex_cfg(48)
    steps = 10
    rho_t = W0[0] + 0.01 * pr.gaussian(5, W0[0].size).reshape(W0[0].shape)
    _, g_ref, _ = misfit_gradient(cfg, W0, rho_t, steps)
    _, g, _ = _gpu_gradient(cfg, W0, rho_t, steps, precision)
    _say(precision, "gradient rel L2", _rel(g, g_ref))
    assert _rel(g, g_ref) <= 1e-3


def test_checkpointing_is_exact():
    """Checkpoint spacing and the overlapped replay (second stream) change
    only the schedule: the gradients agree bit for bit."""
    W0, cfg = _vortex_cfg(32)
    rho_t = W0[0] * 1.001
    g = [_gpu_gradient(cfg, W0, rho_t, 17, "fp64", k)[1] for k in (1, 4, 17)]
    g += [_gpu_gradient(cfg, W0, rho_t, 17, "fp64", k, overlap=False)[1] for k in (4, 5)]
    for x in g[1:]:
        assert np.array_equal(g[0], x)


def _c5(sensor):
    """The adjoint workload: 1024^2 perturbed vortex, misfit against the exact
    density at t = 1, 625 frozen steps of dt = 1/625."""
    n, steps = 1024, 625
    W0, cfg = _vortex_cfg(n)
    cfg["c_fixed"] = cfg["dx"] * steps
    cfg["sensor"] = sensor
    rho_t = pr.vortex(n, t=1.0)[0][0]
    return W0, cfg, rho_t, steps


def _fd_directional(cfg, W0, rho_t, steps, grads, ndir, h=1e-6):
    """Central differences of the FP64 GPU forward along seeded unit directions,
    beside the directional derivatives <g, v> of each gradient in `grads`."""
    from paper_2609_10639_amd import Solver
    from paper_2609_10639_amd.adjoint import Rollout
    run = Rollout(Solver(precision="fp64", **cfg), steps)
    vol = cfg["dx"] ** 2
    rt = torch.tensor(rho_t, device="cuda")

    def Jof(W):
        WT, _ = run.forward(W)
        return float(0.5 * vol * ((WT[0] - rt) ** 2).sum())

    Wd = torch.tensor(W0, device="cuda")
    fds, ads = [], {p: [] for p in grads}
    for m in range(ndir):
        v = pr.gaussian(1000 + m, W0.size).reshape(W0.shape)
        v /= np.linalg.norm(v)
        vd = torch.tensor(v, device="cuda")
        fds.append((Jof(Wd + h * vd) - Jof(Wd - h * vd)) / (2 * h))
        for p, g in grads.items():
            ads[p].append(float((g * v).sum()))
    fds = np.array(fds)
    return fds, {p: np.abs(np.array(a) - fds) / np.abs(fds) for p, a in ads.items()}


def test_full_size_fp64_adjoint_against_finite_differences():
    """FP64 adjoint of the adjoint workload (Sensor B) against central
    differences with h = 1e-6 on 32 seeded directions.  The Ducros gate makes the
    misfit strongly curved, so the difference quotient converges slowly in h:
    measured gaps are ~5e-3 at h = 1e-4, ~1e-4 at 1e-5 and <= 2e-5 at 1e-6,
    hence the bound 1e-4 at h = 1e-6."""
    W0, cfg, rho_t, steps = _c5(2)
    g = _gpu_gradient(cfg, W0, rho_t, steps, "fp64")[1]
    _, rel = _fd_directional(cfg, W0, rho_t, steps, {"fp64": g}, 32)
    _say("fp64 adjoint vs FD: max rel %.2e median %.2e" % (rel["fp64"].max(), np.median(rel["fp64"])))
    assert rel["fp64"].max() <= 1e-4


@pytest.mark.parametrize("precision,tol", [("fp32_mixed", 1e-3), ("fp32", 3e-3)])
def test_full_size_fp32_adjoint_sensor_a(precision, tol):
    """FP32 forms on the adjoint workload with Sensor A (no Ducros gate): the
    gradient against the FP64 adjoint (itself pinned to finite differences)."""
    W0, cfg, rho_t, steps = _c5(1)
    g64 = _gpu_gradient(cfg, W0, rho_t, steps, "fp64")[1]
    g = _gpu_gradient(cfg, W0, rho_t, steps, precision)[1]
    _, rel = _fd_directional(cfg, W0, rho_t, steps, {"fp64": g64, precision: g}, 8)
    _say(precision, "Sensor A: rel L2 vs fp64 %.2e, directional vs FD max %.2e (fp64 %.2e)" % (
        _rel(g, g64), rel[precision].max(), rel["fp64"].max()))
    assert rel["fp64"].max() <= 1e-4
    assert _rel(g, g64) <= tol


_C5_GRADIENTS = {}


def _c5_gradient(precision):
    if precision not in _C5_GRADIENTS:
        W0, cfg, rho_t, steps = _c5(2)
        _C5_GRADIENTS[precision] = _gpu_gradient(cfg, W0, rho_t, steps, precision)[1]
    return _C5_GRADIENTS[precision]


@pytest.mark.parametrize("precision", [
    "fp32_mixed",
    pytest.param("fp32", marks=pytest.mark.xfail(
        strict=False, reason="FP32 arithmetic over 625 forward and 625 adjoint steps: relative L2 1.6e-3 from the "
                             "FP64 gradient; FP32 storage with FP64 arithmetic meets 1e-3 (6.0e-4)"))])
def test_full_size_fp32_adjoint_sensor_b(precision):
    """The adjoint workload as configured (Sensor B): the FP32 gradient against
    the FP64 adjoint (itself pinned to finite differences above)."""
    g64, g = _c5_gradient("fp64"), _c5_gradient(precision)
    _say(precision, "Sensor B: rel L2 vs fp64 %.2e" % _rel(g, g64))
    assert _rel(g, g64) <= 1e-3


@pytest.mark.parametrize("precision,bound", [("fp32_mixed", 2e-3), ("fp32", 5e-3)])
def test_full_size_fp32_adjoint_sensor_b_bound(precision, bound):
    """Regression bound on the measured gaps (6.0e-4 and 1.6e-3)."""
    g64, g = _c5_gradient("fp64"), _c5_gradient(precision)
    assert _rel(g, g64) <= bound
    if precision == "fp32":
        _C5_GRADIENTS.clear()


FP32_STEP_BOUND = {0: 1e-6, 1: 1e-5, 2: 3e-4}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,bc,sensor", [((131, 97), (1, 1, 1, 1), 2), ((131, 97), (0, 0, 1, 1), 2),
                                             ((96, 160), (1, 1, 0, 0), 1), ((70, 70), (0, 0, 0, 0), 0),
                                             ((4, 67), (1, 1, 0, 0), 2), ((5, 7), (0, 0, 0, 0), 2)])
def test_fused_and_multipass_adjoint_step(precision, shape, bc, sensor, monkeypatch):
    """One adjoint step on ragged grids spanning several strips and segments,
    with every boundary mix: the single-march form and the multi-pass form
    against the PyTorch FP64 vector-Jacobian product of the same step at the
    same state (the GPU state, copied out).  Relative Linf bounds: FP64 1e-11;
    FP32 per sensor, from rounding (6e-8) amplified by what the step's adjoint
    does with it: constant beta 1e-6 (measured 1.5e-7), Sensor A 1e-5 (2.9e-6),
    Sensor B 3e-4 (2.5e-5 to 4.1e-5: the transposed sensor at the quadrant
    discontinuities)."""
    tol = 1e-11 if precision == "fp64" else FP32_STEP_BOUND[sensor]
    from oracle.torch_ref import step_vjp
    from paper_2609_10639_amd import Solver
    nx, ny = shape
    n = max(nx, ny)
    W0 = pr.riemann2d(n, 12)[0][:, :ny, :nx].copy()
    W0 = W0 + 1e-3 * np.abs(W0).max(axis=(1, 2), keepdims=True) * pr.gaussian(11, W0.size).reshape(W0.shape)
    cfg = dict(dim=2, nx=nx, ny=ny, dx=1.0 / n, bc=bc, retarget_every=0, c_fixed=4.5, sensor=sensor,
               **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, beta_const=0.9, **pr.IDEAL_AIR.config())
    ref, errs = None, []
    for multipass in ("0", "1"):
        monkeypatch.setenv("VLBM_ADJ_MULTIPASS", multipass)
        s = Solver(precision=precision, **cfg)
        W = torch.tensor(W0, device="cuda")
        f, nrm = s.new_populations(), s.new_norms()
        s.raw_init(W, f, nrm)
        f1, n1 = s.new_populations(), s.new_norms()
        s.raw_step(f, nrm, f1, n1)      # a state with structure
        lam = s.new_populations()
        lam.zero_()   # a cotangent on the cells only, independent of the plane padding
        lam[:, :nx * ny] = torch.tensor(pr.gaussian(12, 16 * nx * ny).reshape(16, nx * ny), dtype=lam.dtype)
        out = s.new_populations()
        out.zero_()
        s.raw_adjoint_step(f1, n1, lam, out)
        torch.cuda.synchronize()
        shp = (4, 4, ny, nx)
        fs = f1[:, :nx * ny].double().cpu().numpy().reshape(shp)
        ls = lam[:, :nx * ny].double().cpu().numpy().reshape(shp)
        g = out[:, :nx * ny].double().cpu().numpy().reshape(shp)
        if ref is None:
            ref = step_vjp(cfg, fs, ls)
        d = np.abs(g - ref).max() / np.abs(ref).max()
        _say("adjoint step", "multi-pass" if multipass == "1" else "fused", precision, shape, bc, sensor,
             "nan cells %d" % int(np.isnan(g).sum()), "rel Linf vs reference %.2e" % d)
        s.close()
        errs.append((np.isfinite(g).all(), d))
    for finite, d in errs:
        assert finite and d <= tol
