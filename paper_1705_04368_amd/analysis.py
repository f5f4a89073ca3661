"""Analysis of MDLG readouts in the paper's terms: velocity moments of a
measured lattice distribution and the consistent space-time discretisation
(Parsa & Wagner, sections "Moments of the equilibrium distribution" and
"Consistent discretizations", with the velocity autocorrelation of the hot
dilute gas from section "Global Equilibrium Distribution").

This is host-side FP64 post-processing of what the library returns
(mdlg_get_f, mdlg_get_shifts, mdlg_get_state): a few hundred numbers per
call, outside the per-step path that the HIP kernels run.

Conventions: a distribution f is indexed by bin i = sum_a (v_a + V)(2V+1)^a
(x fastest), velocities in lattice units per lattice step; a2 is a^2 of
eq. (eqn:a), the per-axis mean squared displacement over (Delta x)^2; u is a
mean velocity in lattice units.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq
from scipy.stats import norm

D2Q9_WEIGHTS = {"rest": ((0, 0), 4.0 / 9.0), "axis": ((1, 0), 1.0 / 9.0),
                "diagonal": ((1, 1), 1.0 / 36.0)}


def lattice_velocities(q, dim):
    """(q, dim) integer lattice velocities of the bins of a length-q
    distribution, q = (2V+1)^dim (axis 0 varies fastest)."""
    side = int(round(q ** (1.0 / dim)))
    if side ** dim != q or side % 2 == 0:
        raise ValueError(f"{q} bins are not a (2V+1)^{dim} window")
    i = np.arange(q)
    return np.stack([(i // side ** ax) % side - side // 2 for ax in range(dim)], axis=1)


def _ramp_mean(x, a):
    """E[(x - Z)_+] for Z ~ N(0, a^2)."""
    return x * norm.cdf(x / a) + a * norm.pdf(x / a)


def equilibrium_factor(y, a2):
    """Per-axis factor of the closed-form equilibrium, eq. (fialpha): the
    chance that a particle displaced by a Gaussian of variance a2 (lattice
    units) from a uniform position in its cell lands y cells away.  The unit
    triangle is the second difference of the ramp, so the factor is
    R(y+1) - 2R(y) + R(y-1) with R(x) = E[(x - Z)_+]."""
    y = np.asarray(y, dtype=np.float64)
    if a2 <= 0:
        return np.maximum(1.0 - np.abs(y), 0.0)
    a = math.sqrt(a2)
    return _ramp_mean(y + 1.0, a) - 2.0 * _ramp_mean(y, a) + _ramp_mean(y - 1.0, a)


def equilibrium(dim, vmax, a2, u=None):
    """Closed-form f_i^eq / rho^eq, eq. (feqfull), on the window |v_a| <= vmax."""
    v = lattice_velocities((2 * vmax + 1) ** dim, dim)
    uu = np.zeros(dim) if u is None else np.asarray(u, dtype=np.float64)
    out = np.ones(len(v))
    for ax in range(dim):
        out = out * equilibrium_factor(v[:, ax] - uu[ax], a2)
    return out


def one_shell(f, dim):
    """The distribution restricted to velocities with all |v_a| <= 1."""
    f = np.asarray(f, dtype=np.float64)
    keep = np.all(np.abs(lattice_velocities(len(f), dim)) <= 1, axis=1)
    return np.where(keep, f, 0.0)


def psi(f, dim, a2, u=None):
    """eq. (eqn:Psi): second moment about u over rho a^2 (dim x dim)."""
    f = np.asarray(f, dtype=np.float64)
    c = lattice_velocities(len(f), dim) - (np.zeros(dim) if u is None else np.asarray(u, float))
    return np.einsum("i,ia,ib->ab", f, c, c) / (f.sum() * a2)


def phi_xxx(f, dim, a2, u=None):
    """eq. (eqn:Phi), xxx component: third moment about u over rho a^3."""
    f = np.asarray(f, dtype=np.float64)
    ux = 0.0 if u is None else float(np.asarray(u, float)[0])
    cx = lattice_velocities(len(f), dim)[:, 0] - ux
    return float(np.dot(f, cx ** 3) / (f.sum() * a2 ** 1.5))


def theta2(f, dim, a2, u=None):
    """eq. (tet2): a^2 Psi_xx."""
    return float(a2 * psi(f, dim, a2, u)[0, 0])


def theta3(f_minus, f_plus, du, dim):
    """eq. (tet3): (1/(3 rho)) d/du_x sum_i f_i v_ix^3, from distributions at
    u_x - du and u_x + du (central difference; rho their mean)."""
    fm = np.asarray(f_minus, dtype=np.float64)
    fp = np.asarray(f_plus, dtype=np.float64)
    vx3 = lattice_velocities(len(fm), dim)[:, 0].astype(np.float64) ** 3
    slope = (np.dot(fp, vx3) - np.dot(fm, vx3)) / (2.0 * du)
    return float(slope / (1.5 * (fm.sum() + fp.sum())))


def m2(f, dim, axis=0):
    """Discrete second moment sum_i f_i v_ia^2 / rho (eq. (eqn:m2) for a
    measured distribution)."""
    f = np.asarray(f, dtype=np.float64)
    va = lattice_velocities(len(f), dim)[:, axis].astype(np.float64)
    return float(np.dot(f, va * va) / f.sum())


def a2_for_weight(vel, w, dim=2, a2_max=4.0):
    """Smallest a^2 with closed-form f_i^eq / rho = w for velocity vel,
    eq. (wif0eqn): bracketed by stepping a^2 up geometrically from 1e-4,
    then solved by Brent's method."""
    vel = np.asarray(vel, dtype=np.float64)

    def g(a2):
        return float(np.prod([equilibrium_factor(vel[ax], a2) for ax in range(dim)])) - w

    lo = 1e-4
    glo = g(lo)
    step = 10 ** (1.0 / 200.0)
    hi = lo
    while hi < a2_max:
        hi2 = hi * step
        if (g(hi2) < 0) != (glo < 0):
            return brentq(g, hi, hi2, xtol=1e-15, rtol=1e-15, maxiter=200)
        hi = hi2
    raise ValueError("weight not reached below a2_max")


def msd_exponential(kT, tau, t, mass=1.0):
    """eq. (vca): per-axis mean squared displacement for the exponential
    velocity autocorrelation (k_B T / m) e^{-t/tau}."""
    x = np.asarray(t, dtype=np.float64) / tau
    return 2.0 * (kT / mass) * tau * tau * (np.expm1(-x) + x)


def dt_for_dx(dx, a2, kT, tau, mass=1.0):
    """Lattice time step at which eq. (vca) gives a^2 (Delta x)^2: the
    consistent Delta t for a given Delta x (Brent's method; eq. (vca) is
    increasing in t)."""
    target = a2 * dx * dx
    hi = tau
    while msd_exponential(kT, tau, hi, mass) < target:
        hi *= 2.0
    return brentq(lambda t: float(msd_exponential(kT, tau, t, mass)) - target, 0.0, hi,
                  xtol=1e-14, rtol=1e-15, maxiter=400)


def fit_tau(t, c, kT, mass=1.0):
    """tau of the exponential velocity autocorrelation: the least-squares
    slope of log(c m / k_B T) against t, through the origin."""
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.asarray(c, dtype=np.float64) / (kT / mass))
    slope = np.dot(t, y) / np.dot(t, t)
    return float(-1.0 / slope)


def vacf_series(system, n_points, md_steps):
    """Measured velocity autocorrelation <v_a(t) v_a(0)> (per axis, averaged
    over particles and axes) at t = k md_steps dt, k = 0..n_points, from the
    system's state read back between plain MD steps.  Returns (k md_steps,
    c) with c[0] = <v_a^2>."""
    d = system.dim
    v0 = system.get_state()["vel"].astype(np.float64)
    steps = [0]
    out = [float(np.mean(np.sum(v0 * v0, axis=1)) / d)]
    for k in range(1, n_points + 1):
        system.step(md_steps)
        v = system.get_state()["vel"].astype(np.float64)
        steps.append(k * md_steps)
        out.append(float(np.mean(np.sum(v * v0, axis=1)) / d))
    return np.array(steps), np.array(out)
