"""The paper's hot dilute gas (the regime of its figures): 2D LJ, N = 100000 in
a 1000 sigma box (rho = 0.1), k_B T = 50, dt = 1e-4, 10 x 10 lattice of
100 sigma, Delta t = 341600 MD steps (34.16 tau), V = 3, with two lattices
drifting at u_x = -/+0.05 for eq. (tet3) (the central difference's O(du^2)
error is below 1e-4 there; a smaller du leaves the sampling noise of one
lattice step larger than the effect).  One lattice step on the GPU, then:

* parity: every analysis quantity of the package (paper_1705_04368_amd.analysis)
  on the GPU's distribution equals the oracle's (independent code) to 1e-12;
* the measured f_i against the closed form eq. (feqfull) at the measured a^2:
  within 3 standard errors plus 2e-3 (the closed form assumes a Gaussian
  displacement, eq. (Pfinal); at Delta t / tau ~ 68 collision times its
  non-Gaussian remainder is of order 1e-3);
* the velocity autocorrelation decays with tau = 0.50 +- 0.05 (the paper's
  fit to the same system), and eq. (vca) with the fitted tau falls short of
  the measured mean squared displacement by at most 10% (the paper ignores
  the 2D long-time tail of the autocorrelation, which only adds to the
  displacement; measured 3.5-6%, the spread coming from the fit of tau on one
  trajectory);
* on the one-shell velocity set theta_2 and theta_3 (eqs. (tet2), (tet3))
  agree with the closed form at the measured a^2 (within 0.01 and 0.015),
  both near 1/3 at this a^2 close to 1/6, and the mean lattice velocity
  vanishes within 3 standard errors.
"""
import math

import numpy as np
import pytest

import oracle.closed_form as cf
import synth
from tests.gpu_util import make_system, say

pytestmark = pytest.mark.gpu

DIM, N, M, DX, KT, DT, STEPS, V, DU = 2, 100000, 10, 100.0, 50.0, 1e-4, 341600, 3, 0.05


def test_hot_dilute_gas_analysis():
    from paper_1705_04368_amd import analysis as an
    from paper_1705_04368_amd import make_config
    say("paper regime: hot dilute gas, one lattice step of 341600 MD steps")
    pos, vel = synth.lj_initial_state(DIM, N, M * DX, KT, seed=2)
    sh = np.zeros((2, 2, DIM))
    sh[0, 1, 0], sh[1, 1, 0] = -DU, DU
    cfg = make_config(DIM, N, M, lattice_dx=DX, dt=DT, md_steps_per_lattice_step=STEPS, vmax=V, kT=KT,
                      shifts=sh)
    sysg = make_system(cfg, pos, vel)
    sysg.step(2000)
    sysg.coarse_grain(1)
    f = sysg.get_f()
    T = f["n_lattice_steps"]
    assert T == 1
    msd = float(np.mean(f["disp_sq"])) / (N * T)
    a2 = msd / DX ** 2
    a = math.sqrt(a2)
    fi = f["f"]
    shf = sysg.get_shifts()
    q = len(fi)
    fm, fp = shf["counts"][0][:q].astype(np.float64), shf["counts"][1][:q].astype(np.float64)
    say(f"  a^2 = {a2:.4f}")

    # parity of the analysis (package against the oracle) on the GPU's data
    for g, gm, gp in ((fi, fm, fp), (cf.one_shell(fi, DIM), cf.one_shell(fm, DIM), cf.one_shell(fp, DIM))):
        np.testing.assert_allclose(an.psi(g, DIM, a2), cf.second_moment_psi(g, DIM, a), rtol=1e-12)
        assert an.phi_xxx(g, DIM, a2) == pytest.approx(cf.third_moment_phi_xxx(g, DIM, a), rel=1e-10,
                                                       abs=1e-14)
        assert an.theta2(g, DIM, a2) == pytest.approx(cf.theta2(g, DIM, a), rel=1e-12)
        assert an.theta3(gm, gp, DU, DIM) == pytest.approx(cf.theta3_from(gm, gp, DU, DIM), rel=1e-12)

    # f_i against the closed form at the measured a^2
    n_samples = N * T
    p = fi / fi.sum()
    ref = cf.feq_over_rho(DIM, V, a)
    se = np.sqrt(np.maximum(p * (1 - p), 1e-12) / n_samples)
    dev = np.abs(p - ref)
    j = int(dev.argmax())
    say(f"  max |f - closed form| {dev[j]:.2e} at bin {j} ({dev[j] / se[j]:.2f} standard errors)")
    assert np.all(dev <= 3 * se + 2e-3)

    # mean lattice velocity and the one-shell temperatures
    v = cf.velocity_grid(DIM, V)
    ubar = (v.T @ p)
    se_u = np.sqrt((v.T.astype(np.float64) ** 2 @ p) / n_samples)
    assert np.all(np.abs(ubar) <= 3 * se_u)
    t2 = cf.theta2(cf.one_shell(fi, DIM), DIM, a)
    t3 = cf.theta3_from(cf.one_shell(fm, DIM), cf.one_shell(fp, DIM), DU, DIM)
    t2_cf = cf.theta2(cf.one_shell(cf.feq_over_rho(DIM, V, a), DIM), DIM, a)
    t3_cf = cf.theta3_from(cf.one_shell(cf.feq_over_rho(DIM, V, a, u=(-DU, 0.0)), DIM),
                           cf.one_shell(cf.feq_over_rho(DIM, V, a, u=(DU, 0.0)), DIM), DU, DIM)
    say(f"  one shell: theta_2 {t2:.4f} (closed form {t2_cf:.4f})  theta_3 {t3:.4f} "
        f"(closed form {t3_cf:.4f})")
    assert abs(t2 - t2_cf) < 0.01 and abs(t3 - t3_cf) < 0.015
    assert abs(t2 - 1 / 3) < 0.03 and abs(t3 - 1 / 3) < 0.03

    # velocity autocorrelation and eq. (vca)
    steps, c = an.vacf_series(sysg, 20, 250)
    t = steps * DT
    tau = cf.fit_tau(t[1:], c[1:], KT)
    pred = cf.msd_exponential_vacf(KT, tau, STEPS * DT)
    say(f"  tau {tau:.4f}; msd measured {msd:.1f}, eq. (vca) {pred:.1f}")
    assert 0.45 <= tau <= 0.55
    assert 0.0 <= msd - pred <= 0.10 * msd
    sysg.close()
