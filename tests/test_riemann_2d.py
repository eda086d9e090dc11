"""Two-dimensional Riemann problems on the CPU (Sec. IV.E-IV.F).

The paper compares its 800^2 runs with a 1000^2 MUSCL reference
(tests/reproduce_paper_tables.py reproduces that comparison; it takes minutes).
Here the oracle is pinned to the one printed fact a small grid can check: the
BZT problem stays in the BZT regime (Gamma < 0 over 99.0 % of the domain).
"""
import numpy as np

from helpers import oracle_for, riemann_bzt_case
from oracle import core
from paper_2609_10639_amd import problems as pr


def test_bzt_riemann_problem_stays_in_the_bzt_regime():
    """BZT four-quadrant problem (Sec. IV.F): the fundamental derivative is
    negative over 99.0 % of the domain at t = 0.35 in the paper's run; the
    oracle at 128^2 gives the same fraction to within half a percent."""
    W0, cfg, t_end = riemann_bzt_case(128)
    o = oracle_for(cfg, W0)
    o.run_to_time(t_end)
    W = o.W()
    c = core.make_config(**pr.BZT_GAS.config())
    e = W[3] / W[0] - 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0] ** 2
    g = np.array([core.gamma_fundamental(c, float(a), float(b)) for a, b in zip(W[0].ravel(), e.ravel())])
    frac = float(np.mean(g < 0))
    print("Gamma < 0 on %.2f %% of the domain" % (100 * frac))
    assert abs(frac - 0.990) < 0.005
