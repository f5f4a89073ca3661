"""Pins for the closed forms of the MDLG equilibrium (CPU only).

eq. (fialpha) is checked against a direct numerical convolution of the wedge
with the Gaussian, against exact sum rules, and against its limits; eq. (vca)
against the integral of eq. (vc) and its ballistic / diffusive limits; the
discrete second moment of eq. (eqn:m2) against the offset of 1/6 the paper
derives; and the paper's printed discretisation (Delta x = 100 sigma,
Delta t = 34.16 tau at k_B T = 50 with tau_v = 0.5) against a^2 ~ 1/6.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import closed_form as cf


@pytest.mark.parametrize("a", [0.05, 0.2, 0.4082, 1.0, 2.5])
@pytest.mark.parametrize("u", [0.0, 0.3, 1.0, -1.7, 2.2])
def test_fialpha_equals_numerical_convolution(a, u):
    def integrand(y):
        return (1.0 - abs(y)) * math.exp(-(u - y) ** 2 / (2 * a * a)) / (math.sqrt(2 * math.pi) * a)
    num, _ = integrate.quad(integrand, -1.0, 1.0, points=[0.0, u], epsabs=1e-14, epsrel=1e-12,
                            limit=200)
    assert float(cf.f_alpha(u, a)) == pytest.approx(num, abs=1e-10)


@pytest.mark.parametrize("a", [0.025, 0.3, 1.0 / math.sqrt(6.0), 1.5])
@pytest.mark.parametrize("u", [0.0, 0.12, 0.5])
def test_fialpha_sum_rules(a, u):
    k = np.arange(-60, 61, dtype=np.float64)
    f = cf.f_alpha(k - u, a)
    assert f.sum() == pytest.approx(1.0, abs=1e-12)      # mass
    assert (k * f).sum() == pytest.approx(u, abs=1e-12)  # exact mean (momentum)
    assert np.all(f >= -1e-15)


def test_fialpha_limits():
    # a -> 0: the bare wedge; the velocity set collapses to the first shell
    # (at the apex the narrow Gaussian shaves off E|y| = a sqrt(2/pi))
    a = 1e-6
    assert float(cf.f_alpha(0.0, a)) == pytest.approx(1.0 - a * math.sqrt(2 / math.pi), abs=1e-12)
    assert float(cf.f_alpha(0.5, a)) == pytest.approx(0.5, abs=1e-12)
    assert float(cf.f_alpha(1.0, a)) == pytest.approx(a / math.sqrt(2 * math.pi), abs=1e-12)
    # large a: Gaussian of variance a^2 + 1/6 (wedge variance) sampled on integers
    a = 6.0
    s2 = a * a + 1.0 / 6.0
    for k in (0, 3, 7):
        g = math.exp(-k * k / (2 * s2)) / math.sqrt(2 * math.pi * s2)
        assert float(cf.f_alpha(k, a)) == pytest.approx(g, rel=2e-3)


def test_feq_products_and_d2q9_regime():
    f = cf.feq_over_rho(2, 1, 1.0 / math.sqrt(6.0))
    v = cf.velocity_grid(2, 1)
    # one shell holds all but the second-shell weight: (1 - 2 f_alpha(2))^2
    assert f.sum() == pytest.approx((1 - 2 * float(cf.f_alpha(2, 1 / math.sqrt(6.0)))) ** 2,
                                    abs=1e-6)
    rest = f[(v[:, 0] == 0) & (v[:, 1] == 0)][0]
    axis = f[(v[:, 0] == 1) & (v[:, 1] == 0)][0]
    diag = f[(v[:, 0] == 1) & (v[:, 1] == 1)][0]
    w0, w1, w5 = cf.D2Q9_WEIGHTS
    # the paper: each of the three D2Q9 matches gives a^2 close to 1/6
    for val, w in ((rest, w0), (axis, w1), (diag, w5)):
        assert val == pytest.approx(w, rel=0.08)

    def root(which, w):
        from scipy.optimize import brentq

        def g(a2):
            ff = cf.feq_over_rho(2, 1, math.sqrt(a2))
            return ff[which] - w
        return brentq(g, 0.05, 0.4)
    idx0 = int(np.where((v[:, 0] == 0) & (v[:, 1] == 0))[0][0])
    idx1 = int(np.where((v[:, 0] == 1) & (v[:, 1] == 0))[0][0])
    idx5 = int(np.where((v[:, 0] == 1) & (v[:, 1] == 1))[0][0])
    roots = [root(idx0, w0), root(idx1, w1), root(idx5, w5)]
    for r in roots:
        assert abs(r - 1.0 / 6.0) < 0.02
    assert max(roots) - min(roots) < 0.01


def test_vca_matches_vacf_integral_and_limits():
    kT, tau = 50.0, 0.5
    for t in (0.01, 0.3, 2.0, 34.16):
        num, _ = integrate.quad(lambda s: 2 * (t - s) * kT * math.exp(-s / tau), 0.0, t,
                                epsabs=1e-12, epsrel=1e-12)
        assert cf.msd_exponential_vacf(kT, tau, t) == pytest.approx(num, rel=1e-9)
    # ballistic limit k_B T t^2, diffusive limit 2 D t - 2 k_B T tau^2 with D = k_B T tau
    t = 1e-3
    assert cf.msd_exponential_vacf(kT, tau, t) == pytest.approx(kT * t * t, rel=1e-3)
    t = 200.0
    assert cf.msd_exponential_vacf(kT, tau, t) == pytest.approx(2 * kT * tau * t - 2 * kT * tau ** 2,
                                                                 rel=1e-12)


def test_printed_discretisation_gives_a2_near_one_sixth():
    # Delta x = 100 sigma, Delta t = 34.16 tau at k_B T = 50, tau_v = 0.5
    a2 = cf.a_squared(cf.msd_exponential_vacf(50.0, 0.5, 34.16), 100.0)
    assert a2 == pytest.approx(1.0 / 6.0, rel=0.02)


def test_second_moment_offsets():
    # uniform start within a cell adds (Delta x)^2 / 12 to the MSD: check by
    # integrating x^2 rho_d(x) of the erf-difference density numerically
    from scipy.special import erf
    D, t, dx = 0.7, 1.3, 1.0

    def rho_d(x):
        s = 2 * math.sqrt(D * t)
        return (erf((x + dx / 2) / s) - erf((x - dx / 2) / s)) / (2 * dx)
    m, _ = integrate.quad(lambda x: x * x * rho_d(x), -40, 40, limit=400)
    assert m == pytest.approx(2 * D * t + dx * dx / 12, rel=1e-9)
    # discrete moment: m2 - a^2 -> 1/6 for large a, smaller for small a
    assert cf.m2_discrete(1.5) - 1.5 ** 2 == pytest.approx(1.0 / 6.0, abs=1e-6)
    assert cf.m2_discrete(0.6) - 0.36 == pytest.approx(1.0 / 6.0, abs=2e-3)
    assert cf.m2_discrete(0.025) - 0.025 ** 2 < 0.05
