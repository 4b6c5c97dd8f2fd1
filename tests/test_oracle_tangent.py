"""Pin of the oracle's tangent-linear model against the definition of the
derivative: central finite differences of the oracle's own forward run,
with a step small enough for O(h^2) truncation and large enough for float64
rounding, agree with the forward-mode directional derivative."""

import numpy as np

from oracle.tangent import CoupledTangent, source_derivatives
from workloads import get_config
from workloads.pulses import knot_values, source_values


def _cfg():
    # differentiation-case molecule model and 64-knot pulse on the tiny grid,
    # field scaled up so that the yield responds visibly
    return get_config("cfg0", n_r=128, j_max=6, pulse="knots", n_knots=64, knot_seed=4,
                      n_steps=120, omega_h=0.10)


def test_tangent_matches_central_differences():
    cfg = _cfg()
    n = cfg.n_steps
    a0 = knot_values(cfg) * 30.0
    rng = np.random.default_rng(7)
    v = rng.standard_normal(cfg.n_knots + 1)
    v[-1] *= cfg.omega * 1e-2          # carrier component in rad/s units
    dS = source_derivatives(cfg, n, knots=a0)
    dsrc = v @ dS
    src0 = source_values(cfg, 0, n, knots=a0)
    tl = CoupledTangent(cfg)
    Y0, dY = tl.run(src0, dsrc)

    def Y_at(eps):
        knots = a0 + eps * v[:-1]
        omega = cfg.omega + eps * v[-1]
        src = source_values(cfg, 0, n, knots=knots, omega=omega)
        t = CoupledTangent(cfg)
        return t.run(src, np.zeros(n))[0]

    h = 1e-3
    fd = (Y_at(h) - Y_at(-h)) / (2 * h)
    assert Y0 > 0 and dY != 0
    assert abs(fd - dY) / abs(dY) < 1e-5, (fd, dY)
