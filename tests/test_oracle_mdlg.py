"""Pins for the oracle's MDLG binning and accumulators (CPU only).

* the worked example of the paper's one-dimensional thought experiment (the
  table of f_0 / f_1 at x = 1..3, t = 1..6 in the figure on lattice momentum),
  reproduced exactly;
* eq. (MDni) evaluated literally with interval indicators on tiny inputs;
* the mass identity N(x,t) = sum_i n_i(x,t) (plus overflow outside the window);
* the lattice momentum summed over sites telescopes to the net change of the
  particles' lattice cells;
* the ideal-gas equilibrium f_i against the wedge form of eq. (fieqW) and the
  Gaussian closed form eq. (feqfull).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import closed_form as cf
import synth


def _bin_index(v, vmax):
    w = 2 * vmax + 1
    return sum((int(v[a]) + vmax) * w ** a for a in range(len(v)))


def test_worked_example_one_particle_table():
    # One particle moving +1/3 of a cell per lattice time step, starting 1.1
    # cells from the origin; cells labelled by floor(position / dx) = 1, 2, 3.
    dx, dim, vmax = 1.0, 2, 1
    lat = oracle.make_lattice(dim, (8, 3), dx, vmax)
    md = oracle.make_md(dim, 1, (8.0, 3.0), dt=0.25, forces_off=True)
    st = oracle.OracleState(md, np.array([[1.1, 1.5]]), np.array([[1.0 / 3.0, 0.0]]),
                            use_cells=False)
    f0, f1 = _bin_index((0, 0), vmax), _bin_index((1, 0), vmax)
    table = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                        "one_particle_table.json")))
    expected = {r["t"]: (r["x"], f0 if r["i"] == 0 else f1) for r in table["rows"]}
    mom_total = 0
    for t in range(1, 7):
        out = st.mdlg(lat, md_per_lattice=4, n_lattice=1)
        A = out["A"].reshape(3, 8, 9)  # [y][x][bin]
        nz = np.argwhere(A > 0)
        assert len(nz) == 1, (t, nz)
        y, x, b = nz[0]
        assert (int(x), int(b)) == expected[t], t
        assert y == 1 and A[y, x, b] == 1
        mom_total += int(out["mom"][:, 2].sum())
    # time-averaged lattice momentum equals the particle velocity 1/3
    assert mom_total / 6 == pytest.approx(1.0 / 3.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_ni_literal_equals_binning(dim):
    rng = np.random.default_rng(7)
    M = (5, 4, 3)[:dim]
    dx, vmax = 2.0, 2
    box = np.array(M, dtype=np.float64) * dx
    lat = oracle.make_lattice(dim, M, dx, vmax)
    n = 60
    now = rng.uniform(-2 * box, 3 * box, size=(n, dim))
    prev = now - rng.normal(0, 1.6 * dx, size=(n, dim))
    # a few positions exactly on cell boundaries
    now[:5] = np.floor(now[:5] / dx) * dx
    prev[5:10] = np.floor(prev[5:10] / dx) * dx
    lit = oracle.ni_literal(lat, dim, prev, now)
    b = oracle.bin_step(lat, dim, prev, now)
    np.testing.assert_array_equal(lit, b["A"])
    # partition of unity: window counts + overflow = N(x, t) per site
    rho, ovf = b["mom"][:, 0], b["mom"][:, 1]
    np.testing.assert_array_equal(b["A"].sum(axis=1).astype(np.int64) + ovf, rho)
    assert rho.sum() == n
    assert ovf.sum() > 0  # some displacements fell outside the window


def _lj_run(dim, seed, n_lattice=6):
    n, box, M = (512, 32.0, 8) if dim == 2 else (512, 10.0, 5)
    dx = box / M
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=seed)
    md = oracle.make_md(dim, n, box, dt=0.005)
    st = oracle.OracleState(md, pos, vel)
    st.run(100, thermo_every=10, kT=1.0)
    lat = oracle.make_lattice(dim, (M,) * dim, dx, 1)
    before = st.unwrapped.copy()
    out = st.mdlg(lat, md_per_lattice=40, n_lattice=n_lattice, per_step_hist=True)
    return st, out, before, dx, n


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_and_momentum_identities_over_a_run(dim):
    st, out, before, dx, n = _lj_run(dim, seed=4)
    T = out["n_lattice"]
    rho, ovf = out["mom"][:, 0], out["mom"][:, 1]
    np.testing.assert_array_equal(out["A"].sum(axis=1).astype(np.int64) + ovf, rho)
    assert rho.sum() == n * T
    assert int(out["hist"].sum()) + int(ovf.sum()) == n * T
    # lattice momentum telescopes: sum over sites and steps of sum_i v_i n_i
    # equals sum over particles of C_j(T) - C_j(0)
    net = (np.floor(st.unwrapped / dx) - np.floor(before / dx)).astype(np.int64).sum(axis=0)
    np.testing.assert_array_equal(out["mom"][:, 2:2 + dim].sum(axis=0), net)
    # continuous displacement sums telescope too
    np.testing.assert_allclose(out["dsum"], (st.unwrapped - before).sum(axis=0), atol=1e-8)


def test_ideal_gas_single_step_matches_wedge_and_closed_form():
    # Uniform positions, Maxwell velocities, no forces: after one lattice time
    # step the expected n_i / N is the mean over particles of the wedge product
    # (eq. (fieqW) with P the empirical displacement distribution); the closed
    # form of eq. (feqfull) is its large-N limit.
    rng = np.random.default_rng(12)
    dim, n, M, dx, kT, vmax = 2, 200000, 16, 4.0, 1.0, 3
    box = M * dx
    dt_lat = 1.6  # a = sqrt(kT) * dt_lat / dx = 0.4
    now0 = rng.uniform(0, box, size=(n, dim))
    vel = synth.maxwell_velocities(dim, n, kT, rng).astype(np.float64)
    prev = now0
    now = now0 + vel * dt_lat
    lat = oracle.make_lattice(dim, (M, M), dx, vmax)
    b = oracle.bin_step(lat, dim, prev, now)
    f_meas = b["A"].sum(axis=0) / n
    f_wedge = cf.feq_finite_sample(dim, vmax, vel * dt_lat / dx)
    f_cf = cf.feq_over_rho(dim, vmax, 0.4)
    se = np.sqrt(f_wedge * (1 - f_wedge) / n) + 1e-12
    assert np.max(np.abs(f_meas - f_wedge) / se) < 5.0
    np.testing.assert_allclose(f_wedge, f_cf, atol=4e-3)
    assert int(b["mom"][:, 1].sum()) == n - int(b["A"].sum())


def test_ideal_gas_trajectory_fi_against_closed_form():
    # forces off, ballistic: a = sqrt(kT/m) Delta t / Delta x
    dim, n, box, M, kT = 2, 2048, 64.0, 16, 1.0
    pos, vel = synth.lj_initial_state(dim, n, box, kT, seed=1)
    md = oracle.make_md(dim, n, box, dt=0.005, forces_off=True)
    st = oracle.OracleState(md, pos, vel, use_cells=False)
    lat = oracle.make_lattice(dim, (M, M), 4.0, 3)
    steps = 320  # Delta t = 1.6, a = 0.4
    out = st.mdlg(lat, md_per_lattice=steps, n_lattice=40)
    f_meas = out["A"].sum(axis=0) / (40 * n)
    f_cf = cf.feq_over_rho(dim, 3, 0.4)
    f_wedge = cf.feq_finite_sample(dim, 3, vel.astype(np.float64) * 1.6 / 4.0)
    big = f_cf > 1e-3
    np.testing.assert_allclose(f_meas[big], f_wedge[big], rtol=0.08)
    np.testing.assert_allclose(f_wedge[big], f_cf[big], rtol=0.08)
    msd = out["dsq"] / (40 * n)
    np.testing.assert_allclose(msd, kT * 1.6 ** 2, rtol=0.08)
