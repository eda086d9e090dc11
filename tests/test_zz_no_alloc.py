"""The allocation-free adjoint step (vlbm_raw_adjoint_step_static) against the
adjoint step that uses the context's scratch, through the C ABI: the same
kernels on the same inputs, so the results agree bit for bit, on two calls in a
row (the second on a smaller grid, so that the static records hold what the
first call left) and on every form; grids beyond the static records and the
multi-pass form are refused."""
import numpy as np
import pytest
import torch

from paper_2609_10639_amd import Solver
from paper_2609_10639_amd import _native as N
from paper_2609_10639_amd import problems as pr

pytestmark = pytest.mark.gpu


def _case(n, precision, sensor=2, step=True):
    W0 = pr.riemann2d(n, 12)[0]
    W0 = W0 + 1e-3 * np.abs(W0).max(axis=(1, 2), keepdims=True) * pr.gaussian(11, W0.size).reshape(W0.shape)
    cfg = dict(dim=2, nx=n, ny=n, dx=1.0 / n, bc=(1, 1, 0, 0), retarget_every=0, c_fixed=4.5, sensor=sensor,
               **pr.SENSOR_2D, eps_theta=pr.EPS_THETA, beta_const=0.9, **pr.IDEAL_AIR.config())
    s = Solver(precision=precision, **cfg)
    W = torch.tensor(W0, device="cuda")
    f, nrm = s.new_populations(), s.new_norms()
    s.raw_init(W, f, nrm)
    f1, n1 = s.new_populations(), s.new_norms()
    if step:
        s.raw_step(f, nrm, f1, n1)   # a state with non-equilibrium content
    else:
        f1, n1 = f, nrm
    lam = s.new_populations()
    lam.zero_()
    lam[:, :n * n] = torch.tensor(pr.gaussian(12, 16 * n * n).reshape(16, n * n), dtype=lam.dtype)
    return s, f1, n1, lam


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_mixed"])
@pytest.mark.parametrize("sensor", [2, 1, 0])
def test_static_adjoint_step_matches(precision, sensor):
    for n in (200, 96):
        s, f, nrm, lam = _case(n, precision, sensor)
        a, b = s.new_populations(), s.new_populations()
        a.zero_()
        b.fill_(7.0)
        s.raw_adjoint_step(f, nrm, lam, a)
        s.raw_adjoint_step_static(f, nrm, lam, b)
        torch.cuda.synchronize()
        cells = n * n
        assert torch.isfinite(a[:, :cells]).all()
        assert torch.equal(a[:, :cells], b[:, :cells]), (n, precision, sensor)
        s.close()


def test_static_adjoint_step_refuses_what_it_cannot_hold(monkeypatch):
    monkeypatch.setenv("VLBM_STRIP_W", "8")   # 64 strips of 8 columns
    monkeypatch.setenv("VLBM_SEG_H", "4")     # 128 segments of 4 rows: 8192 records
    s, f, nrm, lam = _case(512, "fp32", step=False)   # refused on the host, before any launch
    out = s.new_populations()
    with pytest.raises(N.VlbmError) as e:
        s.raw_adjoint_step_static(f, nrm, lam, out)
    assert e.value.status == N.EINVAL and "8192" in str(e.value)
    s.close()
    monkeypatch.delenv("VLBM_STRIP_W")
    monkeypatch.delenv("VLBM_SEG_H")
    monkeypatch.setenv("VLBM_ADJ_MULTIPASS", "1")
    s, f, nrm, lam = _case(64, "fp64", step=False)
    with pytest.raises(N.VlbmError) as e:
        s.raw_adjoint_step_static(f, nrm, lam, s.new_populations())
    assert e.value.status == N.EINVAL
    s.close()
