"""Checks of the seeded input generators (host logic, no GPU)."""
import math

import numpy as np

from paper_2609_10639_amd import problems as pr


def test_splitmix64_reference_outputs():
    # SplitMix64 seeded with 0: published first outputs of the generator
    z = pr.splitmix64(0, np.arange(3))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_and_gaussian_moments():
    u = pr.uniform(1234, 200000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 3e-3
    g = pr.gaussian(42, 200001)
    assert g.size == 200001 and abs(g.mean()) < 1e-2 and abs(g.std() - 1) < 1e-2
    assert np.array_equal(pr.gaussian(42, 10), pr.gaussian(42, 11)[:10])


def test_vortex_is_an_isentropic_radial_equilibrium():
    # Sec. IV.H: dP/dr = rho u_phi^2 / r along the isentrope P = rho^gamma
    r = np.linspace(0.05, 4.0, 400)
    X, Y = 5.0 + r, 5.0 + 0 * r
    rho, u, v, P = pr.isentropic_vortex_primitives(X, Y, background=(0.0, 0.0))
    assert np.allclose(P, rho ** 1.4, rtol=1e-13)
    uphi = v  # on the ray y = y_c the azimuthal direction is +y
    assert np.allclose(uphi, 5.0 / (2 * math.pi) * r * np.exp(0.5 * (1 - r * r)), rtol=1e-13)
    h = 1e-6
    Pp = pr.isentropic_vortex_primitives(X + h, Y, background=(0.0, 0.0))[3]
    Pm = pr.isentropic_vortex_primitives(X - h, Y, background=(0.0, 0.0))[3]
    dPdr = (Pp - Pm) / (2 * h)
    assert np.allclose(dPdr, rho * uphi ** 2 / r, rtol=1e-6, atol=1e-9)


def test_conserved_roundtrip_and_riemann_states():
    W, dx = pr.riemann2d(8, 3)
    assert W.shape == (4, 8, 8) and dx == 1 / 8
    rho = W[0]
    assert rho[7, 7] == 1.5 and rho[0, 0] == 0.138
    P = 0.4 * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / rho)
    assert abs(P[0, 0] - 0.029) < 1e-15 and abs(P[7, 0] - 0.3) < 1e-15


def test_bzt_states_match_paper_quadrants():
    # reduced units of the paper's a = 1, b = 0.3 states (Eq. 49)
    b, a = 0.3, 1.0
    rho_c, P_c = 1 / (3 * b), a / (27 * b * b)
    U = math.sqrt(P_c / rho_c)
    assert abs(pr.BZT_LEFT[0] - 1.0 / rho_c) < 1e-12
    assert abs(pr.BZT_LEFT[1] + 0.15747 / U) < 1e-5
    assert abs(pr.BZT_LEFT[2] - 0.41396 / P_c) < 1e-6
    assert abs(pr.BZT_RIGHT[0] - 0.65 / rho_c) < 1e-12
    assert abs(pr.BZT_RIGHT[2] - 0.36763 / P_c) < 1e-6


def test_riemann_quadrants_cover_odd_grids():
    """Every cell is assigned a quadrant state, also on odd grids where the
    centre lines fall on x = 1/2 and y = 1/2."""
    for n in (7, 8, 131):
        W, _ = pr.riemann2d(n, 12)
        assert np.isfinite(W).all() and (W[0] > 0).all()
