"""Pins for the oracle's analysis of lattice distributions (sections "Moments
of the equilibrium distribution" and "Consistent discretizations"), CPU only.

Each quantity is pinned to facts the paper or the mathematics fixes:
* the discrete second moment m_2 = a^2 + 1/6 once a^2 is not small (the
  paper's figure on m_2), and the exact point-mass identity behind it;
* Psi_xx a^2 equals m_2 for the closed-form equilibrium at rest, Psi is
  diagonal by symmetry, Psi -> 1 for a^2 >> 1;
* Phi_xxx vanishes at u = 0 and decays to 0 for large a^2 at any u;
* theta_2 = theta_3 for large a^2, and theta_3 = 1/3 for the one-shell set at
  small a^2 (v = v^3 there);
* the D2Q9 weights are all matched near a^2 = 1/6;
* the Delta t(Delta x) root-solve reproduces the ballistic and diffusive
  asymptotes of eq. (vca) and the paper's pair Delta x = 100 sigma,
  Delta t = 34.16 tau;
* the exponential-VACF fit recovers tau exactly on exact data.
"""
import math

import numpy as np
import pytest

from oracle import closed_form as cf


@pytest.mark.parametrize("a", [1.0, 2.0, 3.0])
def test_m2_offset_one_sixth(a):
    assert cf.m2_discrete(a) - a * a == pytest.approx(1.0 / 6.0, abs=1e-6)


@pytest.mark.parametrize("y", [0.0, 0.3, 1.25, -2.7])
def test_point_mass_second_moment_identity(y):
    # a particle displaced by exactly y cells, from a uniform position in its
    # cell: its bin probabilities are W(k - y); sum_k k^2 W(k - y) is y^2
    # plus {y}(1 - {y}) (linear interpolation of k^2 between floor and ceil)
    k = np.arange(-6, 7, dtype=np.float64)
    fr = y - math.floor(y)
    assert float(np.sum(k * k * cf.wedge(k - y))) == pytest.approx(y * y + fr * (1 - fr), abs=1e-14)


def test_psi_at_rest_equals_m2_and_is_diagonal():
    for a in (0.5, 1.0, 2.0):
        f = cf.feq_over_rho(2, 16, a)
        psi = cf.second_moment_psi(f, 2, a)
        assert psi[0, 0] * a * a == pytest.approx(cf.m2_discrete(a), rel=1e-9)
        assert psi[1, 1] == pytest.approx(psi[0, 0], rel=1e-12)
        assert abs(psi[0, 1]) < 1e-14
    f = cf.feq_over_rho(2, 40, 6.0)
    assert cf.second_moment_psi(f, 2, 6.0)[0, 0] == pytest.approx(1.0, abs=0.005)


def test_psi_by_hand():
    # three velocities of a 3x3 grid (V = 1): rest, +x, +x+y
    f = np.zeros(9)
    f[4] = 2.0      # v = (0, 0)
    f[5] = 1.0      # v = (1, 0)
    f[8] = 1.0      # v = (1, 1)
    psi = cf.second_moment_psi(f, 2, 0.5, u=(0.25, 0.0))
    # rho = 4; sum f (vx - 0.25)^2 = 2 * 0.0625 + 0.5625 + 0.5625 = 1.25
    assert psi[0, 0] == pytest.approx(1.25 / (4 * 0.25))
    # sum f (vx - 0.25) vy = 0.75 (only v = (1,1)); sum f vy^2 = 1
    assert psi[0, 1] == pytest.approx(0.75 / 1.0)
    assert psi[1, 1] == pytest.approx(1.0 / 1.0)
    assert cf.third_moment_phi_xxx(f, 2, 0.5, u=(0.25, 0.0)) == pytest.approx(
        (2 * (-0.25) ** 3 + 2 * 0.75 ** 3) / (4 * 0.125))


def test_phi_symmetry_and_decay():
    f = cf.feq_over_rho(2, 12, 0.7)
    assert abs(cf.third_moment_phi_xxx(f, 2, 0.7)) < 1e-15
    f = cf.feq_over_rho(2, 24, 2.0, u=(0.3, 0.0))
    assert abs(cf.third_moment_phi_xxx(f, 2, 2.0, u=(0.3, 0.0))) < 1e-6


def test_theta2_theta3_agree_for_large_a2():
    a, du = 1.5, 1e-3
    f0 = cf.feq_over_rho(2, 16, a)
    fm = cf.feq_over_rho(2, 16, a, u=(-du, 0.0))
    fp = cf.feq_over_rho(2, 16, a, u=(du, 0.0))
    t2 = cf.theta2(f0, 2, a)
    t3 = cf.theta3_from(fm, fp, du, 2)
    assert t2 == pytest.approx(a * a + 1.0 / 6.0, rel=1e-6)
    assert t3 == pytest.approx(t2, rel=1e-5)


def test_theta3_one_shell_small_a2():
    a, du = math.sqrt(0.02), 1e-4
    fm = cf.one_shell(cf.feq_over_rho(2, 6, a, u=(-du, 0.0)), 2)
    fp = cf.one_shell(cf.feq_over_rho(2, 6, a, u=(du, 0.0)), 2)
    assert cf.theta3_from(fm, fp, du, 2) == pytest.approx(1.0 / 3.0, abs=1e-3)
    assert np.count_nonzero(fm) == 9


def test_d2q9_weights_matched_near_one_sixth():
    for vel, w in (((0, 0), 4 / 9), ((1, 0), 1 / 9), ((1, 1), 1 / 36)):
        a2 = cf.a2_matching_weight(vel, w)
        a = math.sqrt(a2)
        assert cf.f_alpha(vel[0], a) * cf.f_alpha(vel[1], a) == pytest.approx(w, rel=1e-9)
        assert 0.15 < a2 < 0.2


def test_dt_for_dx_asymptotes_and_the_papers_pair():
    kT, a2 = 50.0, 1.0 / 6.0
    # ballistic: tau >> t, MSD = kT t^2
    t = cf.dt_for_dx(1.0, a2, kT, 1e6)
    assert t == pytest.approx(math.sqrt(a2 / kT), rel=1e-5)
    # diffusive: tau << t, MSD = 2 kT tau (t - tau)
    tau = 1e-3
    t = cf.dt_for_dx(100.0, a2, kT, tau)
    assert t == pytest.approx(a2 * 1e4 / (2 * kT * tau) + tau, rel=1e-9)
    # the figure on u-dependence: Delta x = 100 sigma, Delta t = 34.16 tau at
    # a^2 = 1/6 with the fitted tau = 0.5 (given to two digits)
    assert cf.dt_for_dx(100.0, a2, kT, 0.5) == pytest.approx(34.16, rel=0.02)


def test_fit_tau_recovers_exact_exponential():
    t = np.linspace(0.05, 1.5, 30)
    assert cf.fit_tau(t, cf.vacf_exponential(50.0, 0.5, t), 50.0) == pytest.approx(0.5, rel=1e-12)
