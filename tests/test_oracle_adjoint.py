"""Pins of the reference gradient (oracle/torch_ref.py).

* Its frozen-speed forward equals the C oracle's step by step (two
  independently written implementations of the same map).
* Its autograd gradient matches central finite differences of the C oracle's
  forward along random directions (the derivative's definition).
"""
import numpy as np
import pytest
import torch

from oracle import core
from oracle.torch_ref import Frozen, misfit_gradient
from paper_2609_10639_amd import problems as pr


def _case(n, bc, eos, sensor, noise=1e-3, seed=3):
    if eos == "vdw":
        gas = pr.VDW_REDUCED_CV50
        W = pr.random_admissible_state(2, (n, n), seed=seed, gas=gas, rho_range=(0.55, 0.6), u_amp=0.1,
                                       P_range=(0.85, 0.95))
        c = 4.0
    else:
        gas = pr.IDEAL_AIR
        W, _ = pr.vortex(n)
        W = W + noise * pr.gaussian(seed, W.size).reshape(W.shape)
        c = 4.0 * 10.0 / n * n / 10.0 + 3.0
    cfg = dict(dim=2, nx=n, ny=n, dx=10.0 / n, bc=bc, retarget_every=0, c_fixed=c, sensor=sensor,
               beta_const=0.8, **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, **gas.config())
    return W, cfg


@pytest.mark.parametrize("bc,eos,sensor", [((0, 0, 0, 0), "ideal", 2), ((1, 1, 1, 1), "ideal", 2),
                                           ((1, 1, 0, 0), "vdw", 2), ((0, 0, 0, 0), "ideal", 1),
                                           ((0, 0, 0, 0), "ideal", 0)])
def test_torch_forward_matches_c_oracle(bc, eos, sensor):
    W0, cfg = _case(20, bc, eos, sensor)
    o = core.Oracle(**cfg)
    o.init(W0)
    fr = Frozen(cfg)
    f = fr.init(torch.tensor(W0))
    assert np.abs(f.numpy() - o.f()).max() <= 1e-15 * np.abs(o.f()).max()
    for _ in range(8):
        o.step()
        f = fr.step(f)
        ref = o.f()
        assert np.abs(f.numpy() - ref).max() <= 1e-13 * np.abs(ref).max()


def test_one_dimensional_forward_matches_c_oracle():
    W0, dx = pr.sod(64)
    cfg = dict(dim=1, nx=64, ny=1, dx=dx, bc=(1, 1, 1, 1), retarget_every=0, c_fixed=5.0, sensor=1,
               **pr.SENSOR_1D, eps_theta=pr.EPS_THETA, beta_const=1.0, **pr.IDEAL_AIR.config())
    o = core.Oracle(**cfg)
    o.init(W0)
    fr = Frozen(cfg)
    f = fr.init(torch.tensor(W0))
    for _ in range(10):
        o.step()
        f = fr.step(f)
    assert np.abs(f.numpy() - o.f()).max() <= 1e-13 * np.abs(o.f()).max()


def _J_c_oracle(cfg, W0, rho_t, nsteps):
    o = core.Oracle(**cfg)
    o.init(W0)
    for _ in range(nsteps):
        o.step()
    vol = cfg["dx"] ** 2
    return 0.5 * vol * ((o.W()[0] - rho_t) ** 2).sum()


@pytest.mark.parametrize("bc,eos,sensor", [((0, 0, 0, 0), "ideal", 2), ((1, 1, 1, 1), "ideal", 2),
                                           ((1, 1, 0, 0), "vdw", 2), ((0, 0, 0, 0), "ideal", 0)])
def test_autograd_gradient_matches_finite_differences(bc, eos, sensor):
    n, steps = 16, 6
    W0, cfg = _case(n, bc, eos, sensor)
    rho_t = W0[0] + 0.01 * pr.gaussian(77, n * n).reshape(n, n)
    J, g, _ = misfit_gradient(cfg, W0, rho_t, steps)
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    for m in range(6):
        v = pr.gaussian(1000 + m, W0.size).reshape(W0.shape)
        v /= np.linalg.norm(v)
        h = 1e-6
        fd = (_J_c_oracle(cfg, W0 + h * v, rho_t, steps) - _J_c_oracle(cfg, W0 - h * v, rho_t, steps)) / (2 * h)
        ad = float((g * v).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * np.abs(g).sum() * 1e-3), (m, fd, ad)
