"""Pins for the oracle's binning on displaced and moving lattices (CPU only).

* no displacement and no drift is eq. (MDni) itself: the counts and lattice
  moments equal the plain binning summed over sites;
* lattice-placement averaging: over the K placements a = m / K the lattice
  displacements add up to floor(K y(t)) - floor(K y(t - dt)) per particle and
  axis (Hermite's identity sum_m floor(y + m/K) = floor(K y)), so the averaged
  lattice momentum differs from the continuous displacement by less than 1/K;
* Galilean shift: particles that move by exactly w lattice spacings per
  lattice step all have lattice velocity 0 on the lattice drifting with
  b = -w;
* ideal gas: with drift b = u the histogram of Gaussian displacements of
  uniformly placed particles follows eq. (fialpha) at mean velocity u
  (product over axes), within sampling error.
"""
import numpy as np
import pytest

import oracle
from oracle import closed_form as cf


@pytest.mark.parametrize("dim", [2, 3])
def test_unshifted_equals_plain_binning(dim):
    rng = np.random.default_rng(5 + dim)
    M = (6, 5, 4)[:dim]
    dx, V = 2.0, 2
    lat = oracle.make_lattice(dim, M, dx, V)
    n = 500
    prev = rng.uniform(-10, 30, size=(n, dim))
    now = prev + rng.normal(0, 1.7 * dx, size=(n, dim))
    counts, mom = oracle.bin_shifted(lat, dim, prev, now, np.zeros(dim), np.zeros(dim), 7)
    ref = oracle.bin_step(lat, dim, prev, now)
    np.testing.assert_array_equal(counts[:-1], ref["A"].sum(axis=0).astype(np.int64))
    assert counts[-1] == int(ref["mom"][:, 1].sum()) > 0
    # sum of v over the window equals the momentum columns of the plain binning
    # (which sums v over every particle, as do the shifted moments)
    np.testing.assert_array_equal(mom[:dim], ref["mom"][:, 2:2 + dim].sum(axis=0))


@pytest.mark.parametrize("K", [2, 5, 8])
def test_placement_average_hermite(K):
    rng = np.random.default_rng(K)
    dim, dx = 2, 3.0
    lat = oracle.make_lattice(dim, (7, 7), dx, 7)
    n = 400
    prev = rng.uniform(0, 21, size=(n, dim))
    now = prev + rng.normal(0, 0.8 * dx, size=(n, dim))
    total = np.zeros(dim, dtype=np.int64)
    for m in range(K):
        _, mom = oracle.bin_shifted(lat, dim, prev, now, np.full(dim, m / K), np.zeros(dim), 3)
        total += mom[:dim]
    exact = (np.floor(K * now / dx) - np.floor(K * prev / dx)).sum(axis=0).astype(np.int64)
    np.testing.assert_array_equal(total, exact)
    # the averaged lattice momentum is within n / K of the continuous one
    cont = ((now - prev) / dx).sum(axis=0)
    assert np.all(np.abs(total / K - cont) <= n / K)


def test_galilean_shift_cancels_uniform_motion():
    rng = np.random.default_rng(2)
    dim, dx, w = 2, 4.0, np.array([0.25, -0.375])
    lat = oracle.make_lattice(dim, (8, 8), dx, 2)
    x0 = rng.uniform(0, 32, size=(300, dim))
    for k in range(1, 6):
        prev = x0 + (k - 1) * w * dx
        now = x0 + k * w * dx
        counts, mom = oracle.bin_shifted(lat, dim, prev, now, np.zeros(dim), -w, k)
        W = 5
        centre = (2 + 2 * W)
        assert counts[centre] == 300 and counts.sum() == 300
        np.testing.assert_array_equal(mom, 0)


@pytest.mark.parametrize("u", [0.0, 0.2, 0.45])
def test_ideal_gas_matches_fialpha_at_mean_velocity(u):
    rng = np.random.default_rng(int(100 * u) + 1)
    dim, dx, V = 2, 1.0, 3
    a = 0.55  # standard deviation of the displacement in lattice units
    lat = oracle.make_lattice(dim, (50, 50), dx, V)
    n = 400000
    prev = rng.uniform(0, 50, size=(n, dim))
    now = prev + rng.normal(0, a * dx, size=(n, dim))
    counts, _ = oracle.bin_shifted(lat, dim, prev, now, np.zeros(dim), np.array([u, 0.0]), 4)
    f = counts[:-1] / n
    ref = cf.feq_over_rho(dim, V, a, u=np.array([u, 0.0]))
    se = np.sqrt(ref * (1 - ref) / n)
    z = (f - ref) / np.maximum(se, 1e-12)
    assert np.abs(z).max() < 4.5, np.abs(z).max()
