"""The package's analysis of lattice distributions against the oracle's
(independent implementations of the same definitions), CPU only: closed-form
equilibria at rest and moving, random distributions, and the one-shell
restriction; the root-solves and the VACF fit to solver precision."""
import math

import numpy as np
import pytest

from oracle import closed_form as cf
from paper_1705_04368_amd import analysis as an


@pytest.mark.parametrize("dim,vmax", [(2, 3), (3, 2), (2, 6)])
def test_velocity_order_and_closed_form(dim, vmax):
    q = (2 * vmax + 1) ** dim
    np.testing.assert_array_equal(an.lattice_velocities(q, dim), cf.velocity_grid(dim, vmax))
    for a2, u in ((0.05, None), (1.0 / 6.0, (0.2, -0.1, 0.05)[:dim]), (2.5, (0.45,) + (0.0,) * (dim - 1))):
        np.testing.assert_allclose(an.equilibrium(dim, vmax, a2, u),
                                   cf.feq_over_rho(dim, vmax, math.sqrt(a2), u), rtol=1e-11, atol=1e-15)


def _dists():
    rng = np.random.default_rng(7)
    out = [(2, cf.feq_over_rho(2, 5, 0.6, u=(0.1, 0.0)), 0.36, (0.1, 0.0)),
           (3, cf.feq_over_rho(3, 2, 0.4), 0.16, None)]
    for dim, vmax in ((2, 3), (3, 2)):
        out.append((dim, rng.integers(0, 1000, size=(2 * vmax + 1) ** dim).astype(np.float64), 0.3,
                    tuple(rng.uniform(-0.3, 0.3, size=dim))))
    return out


@pytest.mark.parametrize("case", range(4))
def test_moments_match_oracle(case):
    dim, f, a2, u = _dists()[case]
    a = math.sqrt(a2)
    np.testing.assert_allclose(an.psi(f, dim, a2, u), cf.second_moment_psi(f, dim, a, u), rtol=1e-12,
                               atol=1e-14)
    assert an.phi_xxx(f, dim, a2, u) == pytest.approx(cf.third_moment_phi_xxx(f, dim, a, u), rel=1e-11,
                                                       abs=1e-14)
    assert an.theta2(f, dim, a2, u) == pytest.approx(cf.theta2(f, dim, a, u), rel=1e-12)
    np.testing.assert_array_equal(an.one_shell(f, dim), cf.one_shell(f, dim))
    g = np.roll(f, 3)
    assert an.theta3(f, g, 0.01, dim) == pytest.approx(cf.theta3_from(f, g, 0.01, dim), rel=1e-12)


def test_m2_of_closed_form_matches_oracle_m2():
    for a in (0.3, 1.0, 2.0):
        f = cf.feq_over_rho(2, 16, a)
        assert an.m2(f, 2) == pytest.approx(cf.m2_discrete(a, kmax=16), rel=1e-10)


def test_root_solves_and_fit_match_oracle():
    for name, (vel, w) in an.D2Q9_WEIGHTS.items():
        assert an.a2_for_weight(vel, w) == pytest.approx(cf.a2_matching_weight(vel, w), rel=1e-9), name
    for dx, a2, kT, tau in ((100.0, 1 / 6, 50.0, 0.5), (10.0, 0.3, 1.0, 2.0), (1.0, 0.1, 50.0, 1e3)):
        assert an.dt_for_dx(dx, a2, kT, tau) == pytest.approx(cf.dt_for_dx(dx, a2, kT, tau), rel=1e-10)
        t = np.linspace(0.0, 5 * tau, 7)
        np.testing.assert_allclose(an.msd_exponential(kT, tau, t),
                                   [cf.msd_exponential_vacf(kT, tau, x) for x in t], rtol=1e-13, atol=0)
    rng = np.random.default_rng(3)
    t = np.linspace(0.02, 1.0, 25)
    c = cf.vacf_exponential(50.0, 0.5, t) * (1 + 0.01 * rng.standard_normal(t.size))
    assert an.fit_tau(t, c, 50.0) == pytest.approx(cf.fit_tau(t, c, 50.0), rel=1e-12)
