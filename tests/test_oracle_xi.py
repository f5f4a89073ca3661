"""Pins for the oracle's collision operator Xi_i(x,t) = n_i(x+v_i,t+1) - n_i(x,t)
(eq. Xi), CPU only.

* mass conservation, eq. (Mom0): sum_i Xi_i(x,t) = 0 at every site whenever
  no displacement leaves the velocity window;
* pure streaming: particles that move by a whole lattice vector every lattice
  step (no sub-cell drift) are never "collided": Xi = 0 everywhere;
* the one-particle table of the figure on lattice momentum (the paper's
  printed values, tests/golden/one_particle_table.json): Xi is supported on
  the cell the particle occupies at t, and its lattice momentum
  sum_x sum_i v_i Xi_i(x,t) equals the change P(t+1) - P(t) of the printed
  lattice momentum (sign and time direction of eq. Xi);
* momentum is not conserved in general (the inequality the paper states
  after eq. Mom0): a sub-cell velocity gives nonzero sum_i v_i Xi_i.
"""
import json
import os

import numpy as np
import pytest

import oracle


def _histograms(lat, dim, traj):
    """n_i(x, t) for t = 1 .. len(traj) - 1 from unwrapped positions."""
    return [oracle.bin_step(lat, dim, traj[t - 1], traj[t])["A"].astype(np.int64)
            for t in range(1, len(traj))]


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_conservation_every_site(dim):
    rng = np.random.default_rng(11 + dim)
    M = (6, 5, 4)[:dim]
    dx, V = 2.0, 2
    lat = oracle.make_lattice(dim, M, dx, V)
    n = 400
    box = np.array(M, float) * dx
    x = [rng.uniform(0, box, size=(n, dim))]
    for _ in range(4):
        x.append(x[-1] + rng.uniform(-1.9 * dx, 1.9 * dx, size=(n, dim)))  # |v| <= 2 cells
    hist = _histograms(lat, dim, x)
    for t in range(len(hist) - 1):
        xi = oracle.collision_operator(lat, dim, hist[t], hist[t + 1])
        np.testing.assert_array_equal(xi.sum(axis=1), 0)
        assert np.abs(xi).sum() > 0  # particles did change velocity


@pytest.mark.parametrize("dim", [2, 3])
def test_pure_streaming_has_no_collisions(dim):
    rng = np.random.default_rng(3 + dim)
    M = (7, 6, 5)[:dim]
    dx, V = 1.5, 2
    lat = oracle.make_lattice(dim, M, dx, V)
    n = 300
    box = np.array(M, float) * dx
    x0 = rng.uniform(0, box, size=(n, dim))
    step = rng.integers(-V, V + 1, size=(n, dim)) * dx  # whole lattice vectors
    traj = [x0 + t * step for t in range(5)]
    hist = _histograms(lat, dim, traj)
    for t in range(len(hist) - 1):
        xi = oracle.collision_operator(lat, dim, hist[t], hist[t + 1])
        np.testing.assert_array_equal(xi, 0)


def test_one_particle_table_support_and_momentum():
    table = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                        "one_particle_table.json")))
    rows = {r["t"]: r for r in table["rows"]}
    dim, V, dx = 2, 1, 1.0
    M = (8, 3)
    lat = oracle.make_lattice(dim, M, dx, V)
    # the thought experiment: start 1.1 cells in, move 1/3 cell per lattice step
    traj = [np.array([[1.1 + t / 3.0, 1.5]]) for t in range(7)]
    hist = _histograms(lat, dim, traj)  # t = 1..6
    P = {t: (1 if rows[t]["i"] == 1 else 0) for t in rows}  # printed lattice momentum (x)
    vx = np.array([oracle.bin_velocity(dim, V, i)[0] for i in range((2 * V + 1) ** dim)])
    for t in range(1, 6):
        xi = oracle.collision_operator(lat, dim, hist[t - 1], hist[t]).reshape(M[1], M[0], -1)
        ys, xs = np.nonzero(np.abs(xi).sum(axis=2))
        assert set(xs.tolist()) <= {rows[t]["x"]} and set(ys.tolist()) <= {1}, t
        assert int((xi * vx).sum()) == P[t + 1] - P[t], t


def test_momentum_not_conserved_in_general():
    dim, V = 2, 1
    lat = oracle.make_lattice(dim, (8, 3), 1.0, V)
    traj = [np.array([[1.1 + t / 3.0, 1.5]]) for t in range(5)]
    hist = _histograms(lat, dim, traj)
    vx = np.array([oracle.bin_velocity(dim, V, i)[0] for i in range(9)])
    totals = [int((oracle.collision_operator(lat, dim, hist[t], hist[t + 1]) * vx).sum())
              for t in range(len(hist) - 1)]
    assert any(m != 0 for m in totals)
