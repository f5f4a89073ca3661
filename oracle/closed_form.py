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
    # e^{-x} - 1 + x through expm1: no cancellation for t << tau_v
    return 2.0 * kT * tau_v * tau_v * (math.expm1(-x) + x)


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


# ---------------------------------------------------------------------------
# Moments of a lattice distribution and consistent discretisations
# (sections "Moments of the equilibrium distribution" and "Consistent
# discretizations").  f is indexed like velocity_grid(dim, vmax).

def lattice_velocities_of(f, dim):
    """velocity_grid for a distribution array f of length (2V+1)^dim."""
    q = len(f)
    vmax = int(round(q ** (1.0 / dim))) // 2
    assert (2 * vmax + 1) ** dim == q
    return velocity_grid(dim, vmax)


def second_moment_psi(f, dim, a, u=None):
    """eq. (eqn:Psi): Psi_ab = sum_i f_i (v_ia - u_a)(v_ib - u_b) / (rho a^2),
    rho = sum_i f_i.  Returns the dim x dim matrix."""
    f = np.asarray(f, dtype=np.float64)
    v = lattice_velocities_of(f, dim).astype(np.float64)
    uu = np.zeros(dim) if u is None else np.asarray(u, dtype=np.float64)
    rho = f.sum()
    out = np.zeros((dim, dim))
    for i in range(len(f)):
        c = v[i] - uu
        out += f[i] * np.outer(c, c)
    return out / (rho * a * a)


def third_moment_phi_xxx(f, dim, a, u=None):
    """eq. (eqn:Phi) for alpha = beta = gamma = x:
    sum_i f_i (v_ix - u_x)^3 / (rho a^3)."""
    f = np.asarray(f, dtype=np.float64)
    v = lattice_velocities_of(f, dim).astype(np.float64)
    ux = 0.0 if u is None else float(np.asarray(u, dtype=np.float64)[0])
    total = 0.0
    for i in range(len(f)):
        total += f[i] * (v[i, 0] - ux) ** 3
    return total / (f.sum() * a ** 3)


def one_shell(f, dim):
    """f restricted to the velocities with every |v_a| <= 1 (9 in 2D, 27 in
    3D), the others set to zero."""
    f = np.array(f, dtype=np.float64)
    v = lattice_velocities_of(f, dim)
    f[np.any(np.abs(v) > 1, axis=1)] = 0.0
    return f


def theta2(f, dim, a, u=None):
    """eq. (tet2): theta_2 = a^2 Psi_xx."""
    return a * a * second_moment_psi(f, dim, a, u)[0, 0]


def theta3_from(f_minus, f_plus, du, dim):
    """eq. (tet3): theta_3 = (1 / (3 rho)) d/du_x sum_i f_i v_ix^3, the
    derivative taken as the central difference of two distributions measured
    at u_x -+ du (rho from their mean)."""
    fm = np.asarray(f_minus, dtype=np.float64)
    fp = np.asarray(f_plus, dtype=np.float64)
    v = lattice_velocities_of(fm, dim).astype(np.float64)
    sm = float(np.sum(fm * v[:, 0] ** 3))
    sp = float(np.sum(fp * v[:, 0] ** 3))
    rho = 0.5 * (fm.sum() + fp.sum())
    return (sp - sm) / (2.0 * du) / (3.0 * rho)


def a2_matching_weight(vel, w, dim=2, lo=1e-4, hi=4.0):
    """Smallest a^2 at which the closed-form f_i^eq / rho of one velocity
    equals the lattice Boltzmann weight w, eq. (wif0eqn): the first sign
    change on a logarithmic scan of a^2 from lo, refined by bisection (the
    closed form of a moving velocity first rises from 0, then falls)."""
    vel = np.asarray(vel, dtype=np.float64)

    def g(a2):
        a = math.sqrt(a2)
        return float(np.prod([f_alpha(vel[ax], a) for ax in range(dim)])) - w

    grid = np.geomspace(lo, hi, 2001)
    vals = [g(x) for x in grid]
    k = next(i for i in range(len(grid) - 1) if (vals[i] < 0) != (vals[i + 1] < 0))
    a, b, ga = grid[k], grid[k + 1], vals[k]
    for _ in range(200):
        mid = 0.5 * (a + b)
        gm = g(mid)
        if (gm < 0) == (ga < 0):
            a, ga = mid, gm
        else:
            b = mid
    return 0.5 * (a + b)


def dt_for_dx(dx, a2, kT, tau_v, mass=1.0):
    """Lattice time step Delta t at which the per-axis mean squared
    displacement of eq. (vca) equals a^2 (Delta x)^2 (the consistent
    discretisation for a given Delta x), by bisection (eq. (vca) increases
    monotonically in t)."""
    target = a2 * dx * dx

    def msd(t):
        return msd_exponential_vacf(kT / mass, tau_v, t)

    lo, hi = 0.0, 1.0
    while msd(hi) < target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if msd(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def vacf_exponential(kT, tau_v, t, mass=1.0):
    """The exponential velocity autocorrelation of the hot dilute gas,
    <v_a(t) v_a(0)> = (k_B T / m) exp(-t / tau_v)."""
    return kT / mass * np.exp(-np.asarray(t, dtype=np.float64) / tau_v)


def fit_tau(t, vacf, kT, mass=1.0):
    """tau_v of the exponential fit: least squares of log(vacf m / k_B T) =
    -t / tau_v through the origin."""
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.asarray(vacf, dtype=np.float64) * mass / kT)
    return -float(np.sum(t * t) / np.sum(t * y))
