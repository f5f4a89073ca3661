"""Pins for the oracle's molecular dynamics (CPU only).

The oracle's forces and integrator are checked against facts fixed by the
mathematics rather than against themselves: textbook two-body values of the
LJ potential, the force as minus the gradient of the energy (finite
differences of the oracle's energy), Newton's third law, the free-flight closed
form, time reversibility, and momentum / energy conservation of velocity
Verlet.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def test_lj_textbook_values():
    # V(sigma) = 0, minimum V = -eps at r = 2^(1/6) sigma, where the force vanishes
    assert oracle.lj_potential(1.0) == 0.0
    rmin = 2.0 ** (1.0 / 6.0)
    assert oracle.lj_potential(rmin) == pytest.approx(-1.0, abs=1e-14)
    assert abs(oracle.lj_force_over_r(rmin)) < 1e-13
    # |F(sigma)| = 24 eps / sigma, repulsive
    assert oracle.lj_force_over_r(1.0) * 1.0 == pytest.approx(24.0, rel=1e-15)
    # scaling with eps and sigma: V(r; eps, sigma) = eps V(r/sigma; 1, 1)
    assert oracle.lj_potential(2.6, eps=1.7, sigma=1.3) == pytest.approx(
        1.7 * oracle.lj_potential(2.6 / 1.3), rel=1e-14)
    # attractive beyond the minimum
    assert oracle.lj_force_over_r(1.5) < 0


def test_force_is_minus_energy_gradient_pair():
    # g(r) r = -dV/dr, checked by a central difference of V alone
    for r in (0.95, 1.05, 1.3, 2.0, 2.4):
        h = 1e-6
        dvdr = (oracle.lj_potential(r + h) - oracle.lj_potential(r - h)) / (2 * h)
        assert oracle.lj_force_over_r(r) * r == pytest.approx(-dvdr, rel=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_forces_are_minus_gradient_of_total_energy(dim):
    n, box = 24 if dim == 2 else 40, 8.0
    pos, _ = synth.lj_initial_state(dim, n, box, 1.0, seed=11, r_min=0.85)
    x = pos.astype(np.float64)
    md = oracle.make_md(dim, n, box, rc=2.5)
    acc, _ = oracle.forces(md, x, brute=True)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(12):
        i, a = int(rng.integers(n)), int(rng.integers(dim))
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        _, ep = oracle.forces(md, xp, brute=True)
        _, em = oracle.forces(md, xm, brute=True)
        # energy shift is a constant per pair inside the cutoff; pairs crossing
        # r_c are absent for this tiny displacement with overwhelming likelihood
        assert acc[i, a] == pytest.approx(-(ep - em) / (2 * h), rel=2e-5, abs=2e-5)


@pytest.mark.parametrize("dim", [2, 3])
def test_cells_equal_brute_force_and_newton3(dim):
    n, box = (300, 20.0) if dim == 2 else (500, 10.0)
    pos, _ = synth.lj_initial_state(dim, n, box, 1.0, seed=3)
    x = pos.astype(np.float64)
    md = oracle.make_md(dim, n, box, rc=2.5)
    ab, eb = oracle.forces(md, x, brute=True)
    ac, ec = oracle.forces(md, x, brute=False)
    np.testing.assert_allclose(ac, ab, rtol=1e-12, atol=1e-10)
    assert ec == pytest.approx(eb, rel=1e-12)
    np.testing.assert_allclose(ab.sum(axis=0), 0.0, atol=1e-9)


@pytest.mark.parametrize("dim,n,box", [(2, 300, 20.0), (3, 500, 10.0), (2, 20, 6.0)])
def test_sampled_forces_equal_brute_force(dim, n, box):
    # the sampled evaluation (used at sizes too large for a full one) against
    # the brute-force sum over all partners; the last case has fewer than 3
    # cells per axis and takes the all-pairs branch
    pos, _ = synth.lj_initial_state(dim, n, box, 1.0, seed=9, r_min=0.8)
    x = pos.astype(np.float64)
    md = oracle.make_md(dim, n, box, rc=2.5)
    ab, _ = oracle.forces(md, x, brute=True)
    idx = np.random.default_rng(4).choice(n, size=n // 3, replace=False)
    np.testing.assert_allclose(oracle.forces_subset(md, x, idx), ab[idx], rtol=1e-12, atol=1e-10)
    assert np.abs(ab[idx]).max() > 0.1  # nonzero forces were compared


def test_minimum_image_pair_across_boundary():
    # two particles 1.1 sigma apart across the periodic boundary
    md = oracle.make_md(2, 2, 10.0, rc=2.5)
    x = np.array([[0.3, 5.0], [9.2, 5.0]])
    acc, _ = oracle.forces(md, x, brute=True)
    r = 1.1
    g = oracle.lj_force_over_r(r)
    # particle 0 sits at +x of particle 1's image: F_0 = g * (+r) along x
    assert acc[0, 0] == pytest.approx(g * r, rel=1e-12)
    assert acc[1, 0] == pytest.approx(-g * r, rel=1e-12)
    assert abs(acc[0, 1]) < 1e-15


def test_free_flight_closed_form_with_images():
    dim, n, box = 2, 50, 12.0
    pos, vel = synth.lj_initial_state(dim, n, box, 4.0, seed=9)
    md = oracle.make_md(dim, n, box, dt=0.01, forces_off=True)
    st = oracle.OracleState(md, pos, vel, use_cells=False)
    st.run(1000)
    expect = pos.astype(np.float64) + vel.astype(np.float64) * 10.0
    np.testing.assert_allclose(st.unwrapped, expect, rtol=0, atol=1e-10)
    assert np.all(st.x >= 0) and np.all(st.x < box)
    assert np.abs(st.img).max() >= 1  # some particles crossed the boundary


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_verlet_reversible_and_conservative(dim):
    n, box = (256, 22.63) if dim == 2 else (256, 7.5)
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=21)
    md = oracle.make_md(dim, n, box, dt=0.002)
    st = oracle.OracleState(md, pos, vel)
    ke0, p0 = st.kinetics()
    _, ep0 = oracle.forces(md, st.x)
    st.run(200)
    ke1, p1 = st.kinetics()
    _, ep1 = oracle.forces(md, st.x)
    np.testing.assert_allclose(p1, p0, atol=1e-10)
    assert abs((ke1 + ep1) - (ke0 + ep0)) < 5e-3 * (abs(ke0) + abs(ep0))
    # reverse: negate velocities and integrate back
    st.v *= -1.0
    st.acc, _ = oracle.forces(md, st.x)
    st.run(200)
    np.testing.assert_allclose(st.unwrapped, pos.astype(np.float64), atol=1e-7)
    np.testing.assert_allclose(-st.v, vel.astype(np.float64), atol=1e-7)


def test_thermostat_sets_temperature():
    dim, n, box = 2, 400, 28.28
    pos, vel = synth.lj_initial_state(dim, n, box, 3.0, seed=2)
    md = oracle.make_md(dim, n, box, dt=0.005)
    st = oracle.OracleState(md, pos, vel)
    st.run(100, thermo_every=10, kT=1.0)
    ke, _ = st.kinetics()
    assert 2 * ke / (dim * (n - 1)) == pytest.approx(1.0, rel=1e-12)


def test_jittered_grid_min_distance():
    pos, vel = synth.lj_initial_state(2, 2048, 64.0, 1.0, seed=1)
    x = pos.astype(np.float64)
    d = x[:, None, :] - x[None, :, :]
    d -= 64.0 * np.round(d / 64.0)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(x)) * 1e9
    assert r.min() >= 0.8 - 1e-5
    assert np.all(x >= 0) and np.all(x < 64.0)
    assert abs(float(np.sum(vel.astype(np.float64) ** 2)) / (2 * 2047) - 1.0) < 1e-5
    assert math.isclose(float(vel.astype(np.float64).mean(0)[0]), 0.0, abs_tol=1e-6)
