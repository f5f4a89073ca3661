"""Closed forms of the MDLG equilibrium theory -- TEST INFRASTRUCTURE ONLY.

Part of the oracle: only the tests, the smoke check and the CPU-baseline leg of
the bench use it.  Written from the paper (Parsa & Wagner, "Lattice Gas with
Molecular Dynamics Collision Operator"), section "Global Equilibrium
Distribution" and section "Consistent discretizations".

Notation follows the paper: ``a`` is the root-mean-square per-axis displacement
in lattice units, eq. (eqn:a); ``u`` is the mean velocity in lattice units per
lattice time step (the paper writes u Delta t in physical units inside P_alpha
and u_alpha in lattice units inside f_{i,alpha}; the lattice-unit reading is
used here).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def f_alpha(u, a):
    """Per-axis factor f_{i,alpha}^eq of eq. (fialpha).

    It is the unit triangle ("wedge" W of eq. (fieqW), in lattice units)
    convolved with a centred Gaussian of standard deviation ``a``, evaluated at
    u = v_{i,alpha} - u_alpha.  Vectorised over ``u``.
    """
    u = np.asarray(u, dtype=np.float64)
    a = float(a)
    if a <= 0.0:
        return np.clip(1.0 - np.abs(u), 0.0, None)
    norm = a / math.sqrt(2.0 * math.pi)
    s = math.sqrt(2.0) * a
    gauss = (np.exp(-((u - 1.0) ** 2) / (2 * a * a))
             - 2.0 * np.exp(-(u ** 2) / (2 * a * a))
             + np.exp(-((u + 1.0) ** 2) / (2 * a * a)))
    lin = ((u - 1.0) / 2.0 * (erf((u - 1.0) / s) - erf(u / s))
           + (u + 1.0) / 2.0 * (erf((u + 1.0) / s) - erf(u / s)))
    return norm * gauss + lin


def velocity_grid(dim, vmax):
    """Lattice velocities of the window |v_alpha| <= vmax, in the bin order
    i = sum_alpha (v_alpha + V) (2V+1)^alpha (x fastest).  Shape (Q, dim)."""
    w = 2 * vmax + 1
    q = w ** dim
    idx = np.arange(q)
    out = np.empty((q, dim), dtype=np.int64)
    for ax in range(dim):
        out[:, ax] = (idx // (w ** ax)) % w - vmax
    return out


def feq_over_rho(dim, vmax, a, u=None):
    """f_i^eq / rho^eq of eq. (feqfull) on the window |v_alpha| <= vmax.

    ``a`` may be a scalar (isotropic) or a per-axis sequence; ``u`` is the mean
    velocity per axis in lattice units (default 0)."""
    v = velocity_grid(dim, vmax)
    a_ax = np.broadcast_to(np.asarray(a, dtype=np.float64), (dim,))
    u_ax = np.zeros(dim) if u is None else np.asarray(u, dtype=np.float64)
    out = np.ones(v.shape[0])
    for ax in range(dim):
        out *= f_alpha(v[:, ax] - u_ax[ax], a_ax[ax])
    return out


def a_squared(msd_axis, dx):
    """eq. (eqn:a): a^2 = <(delta x_alpha)^2> / (Delta x)^2."""
    return msd_axis / (dx * dx)


def msd_ballistic(kT, mass, dt_lat):
    """Ballistic per-axis mean squared displacement k_B T (Delta t)^2 / m
    (Maxwell-Boltzmann velocities, no collisions)."""
    return kT / mass * dt_lat * dt_lat


def msd_exponential_vacf(kT, tau_v, t):
    """eq. (vca): per-axis MSD for an exponentially decaying velocity
    autocorrelation k_B T exp(-t/tau_v), 2 k_B T tau_v^2 (e^{-t/tau_v} + t/tau_v - 1)."""
    x = t / tau_v
    return 2.0 * kT * tau_v * tau_v * (math.exp(-x) + x - 1.0)


def wedge(y):
    """Per-axis wedge W_alpha in lattice units: (1 - |y|) for |y| < 1, else 0."""
    y = np.asarray(y, dtype=np.float64)
    return np.clip(1.0 - np.abs(y), 0.0, None)


def feq_finite_sample(dim, vmax, disp):
    """Expected f_i / rho for a finite set of particles with fixed per-lattice-step
    displacements ``disp`` (shape (N, dim), lattice units) and positions uniform
    within their cell: the mean over particles of prod_alpha W(v_{i,alpha} - d_alpha)
    (eq. (fieqW) with P a sum of point masses)."""
    v = velocity_grid(dim, vmax)
    disp = np.asarray(disp, dtype=np.float64)
    out = np.ones((v.shape[0], disp.shape[0]))
    for ax in range(dim):
        out *= wedge(v[:, ax][:, None] - disp[:, ax][None, :])
    return out.mean(axis=1)


def m2_discrete(a, kmax=None):
    """Discrete second moment of eq. (eqn:m2) in lattice units:
    sum_k k^2 * (probability that the displacement falls in bin k), where the
    displacement density is the uniform in-cell start convolved with the
    Gaussian of variance a^2; that bin probability is f_alpha(k, a)."""
    if kmax is None:
        kmax = int(math.ceil(12 * a + 4))
    k = np.arange(-kmax, kmax + 1, dtype=np.float64)
    return float(np.sum(k * k * f_alpha(k, a)))


D2Q9_WEIGHTS = (4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0)
"""D2Q9 lattice Boltzmann weights w_0, w_{1-4}, w_{5-8} (section "Relation of
MDLG equilibrium functions to lattice Boltzmann equilibria")."""
