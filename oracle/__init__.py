"""FP64 CPU oracle for the MDLG hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C oracle
(``mdlg_oracle.c``) with numpy arrays and re-exports the closed forms of
``closed_form``.  It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import closed_form  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc_mdlg.so")
_lib = None


class OrcMD(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("box", C.c_double * 3),
                ("eps", C.c_double), ("sigma", C.c_double), ("mass", C.c_double),
                ("rc", C.c_double), ("forces_off", C.c_int), ("dt", C.c_double)]


class OrcLattice(C.Structure):
    _fields_ = [("M", C.c_int * 3), ("dx", C.c_double), ("V", C.c_int)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    dp, ip, up, lp = P(C.c_double), P(C.c_int32), P(C.c_uint64), P(C.c_int64)
    lib.orc_lj_potential.restype = C.c_double
    lib.orc_lj_potential.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.orc_lj_force_over_r.restype = C.c_double
    lib.orc_lj_force_over_r.argtypes = [C.c_double, C.c_double, C.c_double]
    for name in ("orc_forces_brute", "orc_forces_cells"):
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = [P(OrcMD), dp, dp, dp]
    lib.orc_forces_subset.restype = C.c_int
    lib.orc_forces_subset.argtypes = [P(OrcMD), dp, ip, C.c_int, dp]
    lib.orc_vv.restype = C.c_int
    lib.orc_vv.argtypes = [P(OrcMD), dp, ip, dp, dp, C.c_long, P(C.c_long), C.c_int,
                           C.c_double, C.c_int]
    lib.orc_equilibrate.restype = C.c_int
    lib.orc_equilibrate.argtypes = lib.orc_vv.argtypes
    lib.orc_num_moments.restype = C.c_int
    lib.orc_num_moments.argtypes = [C.c_int]
    lib.orc_bin.restype = C.c_int
    lib.orc_bin.argtypes = [P(OrcLattice), C.c_int, C.c_int, dp, dp, up, lp, dp, dp]
    lib.orc_ni_literal.restype = C.c_int
    lib.orc_ni_literal.argtypes = [P(OrcLattice), C.c_int, C.c_int, dp, dp, up]
    lib.orc_mdlg_run.restype = C.c_int
    lib.orc_mdlg_run.argtypes = [P(OrcMD), P(OrcLattice), C.c_int, C.c_long, dp, ip, dp,
                                 dp, P(C.c_long), C.c_int, up, lp, dp, dp, up]
    lib.orc_kinetics.restype = None
    lib.orc_kinetics.argtypes = [P(OrcMD), dp, dp, dp]
    lib.orc_pair_terms.restype = C.c_int
    lib.orc_pair_terms.argtypes = [P(OrcMD), dp, dp, dp, dp, dp]
    lib.orc_adjoint.restype = C.c_int
    lib.orc_adjoint.argtypes = [P(OrcMD), dp, dp, C.c_int, C.c_int, dp, dp, dp, dp, dp]
    lib.orc_window_loss.restype = C.c_int
    lib.orc_window_loss.argtypes = [P(OrcMD), dp, dp, C.c_int, C.c_int, dp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_moments(dim):
    return int(_load().orc_num_moments(dim))


def lj_potential(r, eps=1.0, sigma=1.0):
    return float(_load().orc_lj_potential(float(r), eps, sigma))


def lj_force_over_r(r, eps=1.0, sigma=1.0):
    return float(_load().orc_lj_force_over_r(float(r), eps, sigma))


def make_md(dim, n, box, eps=1.0, sigma=1.0, mass=1.0, rc=2.5, dt=0.005, forces_off=False):
    p = OrcMD()
    p.dim = dim
    p.n = n
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (dim,))
    for a in range(3):
        p.box[a] = float(b[a]) if a < dim else 1.0
    p.eps, p.sigma, p.mass, p.rc, p.dt = eps, sigma, mass, rc, dt
    p.forces_off = int(bool(forces_off))
    return p


def make_lattice(dim, M, dx, vmax):
    L = OrcLattice()
    m = np.broadcast_to(np.asarray(M, dtype=np.int64), (dim,))
    for a in range(3):
        L.M[a] = int(m[a]) if a < dim else 1
    L.dx = float(dx)
    L.V = int(vmax)
    return L


def forces(md, x, brute=False):
    """Accelerations a_i = F_i / m (FP64) and the shifted potential energy."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    ep = C.c_double(0.0)
    f = _load().orc_forces_brute if brute else _load().orc_forces_cells
    _check(f(C.byref(md), _dp(x), _dp(acc), C.byref(ep)), "forces")
    return acc, ep.value


def forces_subset(md, x, idx):
    """Accelerations of the particles idx only (rows in the order of idx),
    each summed over all its partners as in forces(): for sampled checks of
    systems too large for a full evaluation."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    acc = np.zeros((idx.shape[0], x.shape[1]))
    _check(_load().orc_forces_subset(C.byref(md), _dp(x), _ip(idx), int(idx.shape[0]), _dp(acc)),
           "forces_subset")
    return acc


class OracleState:
    """Particle state of the FP64 oracle: wrapped positions in [0, L), image
    counters, velocities and the accelerations at the current positions."""

    def __init__(self, md, pos, vel, img=None, use_cells=True):
        self.md = md
        self.use_cells = int(bool(use_cells))
        self.x = np.ascontiguousarray(pos, dtype=np.float64).copy()
        self.v = np.ascontiguousarray(vel, dtype=np.float64).copy()
        self.img = (np.zeros(self.x.shape, dtype=np.int32) if img is None
                    else np.ascontiguousarray(img, dtype=np.int32).copy())
        self.step = C.c_long(0)
        self.acc, _ = forces(md, self.x, brute=not use_cells)

    @property
    def unwrapped(self):
        box = np.array([self.md.box[a] for a in range(self.md.dim)])
        return self.x + self.img * box

    def run(self, nsteps, thermo_every=0, kT=0.0):
        _check(_load().orc_vv(C.byref(self.md), _dp(self.x), _ip(self.img), _dp(self.v),
                              _dp(self.acc), int(nsteps), C.byref(self.step),
                              int(thermo_every), float(kT), self.use_cells), "vv")

    def kinetics(self):
        ke = C.c_double(0.0)
        mom = np.zeros(3)
        _load().orc_kinetics(C.byref(self.md), _dp(self.v), C.byref(ke), _dp(mom))
        return ke.value, mom[: self.md.dim].copy()

    def mdlg(self, lattice, md_per_lattice, n_lattice, per_step_hist=False):
        """Run n_lattice lattice steps; returns a dict of accumulators."""
        dim = self.md.dim
        nsite = int(np.prod([lattice.M[a] for a in range(dim)]))
        q = (2 * lattice.V + 1) ** dim
        nm = num_moments(dim)
        A = np.zeros((nsite, q), dtype=np.uint64)
        mom = np.zeros((nsite, nm), dtype=np.int64)
        dsum = np.zeros(dim)
        dsq = np.zeros(dim)
        hist = np.zeros((n_lattice, q), dtype=np.uint64) if per_step_hist else None
        hp = _up(hist) if per_step_hist else C.cast(None, C.POINTER(C.c_uint64))
        _check(_load().orc_mdlg_run(C.byref(self.md), C.byref(lattice), int(md_per_lattice),
                                    int(n_lattice), _dp(self.x), _ip(self.img), _dp(self.v),
                                    _dp(self.acc), C.byref(self.step), self.use_cells,
                                    _up(A), _lp(mom), _dp(dsum), _dp(dsq), hp), "mdlg_run")
        return {"A": A, "mom": mom, "dsum": dsum, "dsq": dsq, "hist": hist,
                "n_lattice": n_lattice, "n_sites": nsite}


def bin_step(lattice, dim, xu_prev, xu_now):
    """One lattice step of binning on given unwrapped FP64 positions."""
    xu_prev = np.ascontiguousarray(xu_prev, dtype=np.float64)
    xu_now = np.ascontiguousarray(xu_now, dtype=np.float64)
    n = xu_now.shape[0]
    nsite = int(np.prod([lattice.M[a] for a in range(dim)]))
    q = (2 * lattice.V + 1) ** dim
    A = np.zeros((nsite, q), dtype=np.uint64)
    mom = np.zeros((nsite, num_moments(dim)), dtype=np.int64)
    dsum = np.zeros(dim)
    dsq = np.zeros(dim)
    _check(_load().orc_bin(C.byref(lattice), dim, n, _dp(xu_prev), _dp(xu_now), _up(A),
                           _lp(mom), _dp(dsum), _dp(dsq)), "bin")
    return {"A": A, "mom": mom, "dsum": dsum, "dsq": dsq}


def ni_literal(lattice, dim, xu_prev, xu_now):
    """eq. (MDni) evaluated literally with interval indicators (tiny inputs)."""
    xu_prev = np.ascontiguousarray(xu_prev, dtype=np.float64)
    xu_now = np.ascontiguousarray(xu_now, dtype=np.float64)
    n = xu_now.shape[0]
    nsite = int(np.prod([lattice.M[a] for a in range(dim)]))
    q = (2 * lattice.V + 1) ** dim
    out = np.zeros((nsite, q), dtype=np.uint64)
    _check(_load().orc_ni_literal(C.byref(lattice), dim, n, _dp(xu_prev), _dp(xu_now),
                                  _up(out)), "ni_literal")
    return out


def pair_terms(md, x, lam=None):
    """Accelerations, their sigma derivative and the Jacobian-vector product
    J lam (J = d a / d x) on wrapped FP64 positions."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    acc, dacc, jl = np.zeros_like(x), np.zeros_like(x), np.zeros_like(x)
    lp = _dp(np.ascontiguousarray(lam, dtype=np.float64)) if lam is not None else None
    keep = lam
    _check(_load().orc_pair_terms(C.byref(md), _dp(x), lp, _dp(acc), _dp(dacc),
                                  _dp(jl) if lam is not None else None), "pair_terms")
    del keep
    return acc, dacc, (jl if lam is not None else None)


LOSSES = {"msd": 0, "mean_x": 1}


def adjoint(md, x0, v0, window, loss):
    """Loss of the displacement over `window` velocity-Verlet steps and its
    gradients with respect to eps, sigma, v0 and x0 (FP64 reverse sweep)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    L, ge, gs = C.c_double(0), C.c_double(0), C.c_double(0)
    gv, gx = np.zeros_like(v0), np.zeros_like(x0)
    _check(_load().orc_adjoint(C.byref(md), _dp(x0), _dp(v0), int(window), LOSSES[loss],
                               C.byref(L), C.byref(ge), C.byref(gs), _dp(gv), _dp(gx)), "adjoint")
    return {"L": L.value, "eps": ge.value, "sigma": gs.value, "v0": gv, "x0": gx}


def window_loss(md, x0, v0, window, loss):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    L = C.c_double(0)
    _check(_load().orc_window_loss(C.byref(md), _dp(x0), _dp(v0), int(window), LOSSES[loss],
                                   C.byref(L)), "window_loss")
    return L.value


def bin_velocity(dim, vmax, i):
    """Lattice velocity of bin i (i = sum_a (v_a + V) (2V + 1)^a, x fastest)."""
    w = 2 * vmax + 1
    return tuple((i // w ** a) % w - vmax for a in range(dim))


def collision_operator(lattice, dim, n_t, n_next):
    """The MDLG collision operator of eq. (Xi),
        Xi_i(x, t) = n_i(x + v_i, t + 1) - n_i(x, t),
    from the occupation numbers of eq. (MDni) at two consecutive lattice times
    (arrays [n_sites][Q], site index x fastest) on the periodic lattice.
    Returns int64 [n_sites][Q]."""
    M = [int(lattice.M[a]) for a in range(dim)]
    V = int(lattice.V)
    Q = (2 * V + 1) ** dim
    grid = tuple(reversed(M))  # numpy axes (z,) y, x
    now = np.asarray(n_t, dtype=np.int64).reshape(grid + (Q,))
    nxt = np.asarray(n_next, dtype=np.int64).reshape(grid + (Q,))
    xi = np.zeros_like(now)
    for i in range(Q):
        v = bin_velocity(dim, V, i)
        # shifted[x] = n_i(x + v_i, t + 1): roll by -v along every axis
        shifted = nxt[..., i]
        for a in range(dim):
            shifted = np.roll(shifted, -v[a], axis=dim - 1 - a)
        xi[..., i] = shifted - now[..., i]
    return xi.reshape(-1, Q)


def bin_shifted(lattice, dim, xu_prev, xu_now, a, b, k):
    """eq. (MDni) on a displaced, moving lattice, summed over sites: at lattice
    time k a particle at x is in cell floor(x / dx + a + b k) per axis (a, b
    in lattice spacings; b = u bins the Galilean-transformed positions
    x + u t).  Returns (counts [Q + 1]: window bins then the overflow,
    moments [d + d(d+1)/2]: sum of v_a over all particles, then v_a v_b)."""
    dx = float(lattice.dx)
    V = int(lattice.V)
    W = 2 * V + 1
    Q = W ** dim
    a = np.asarray(a, dtype=np.float64).reshape(dim)
    b = np.asarray(b, dtype=np.float64).reshape(dim)
    y_now = np.asarray(xu_now, dtype=np.float64) / dx
    y_prev = np.asarray(xu_prev, dtype=np.float64) / dx
    now = a + b * float(k)
    before = a + b * (float(k) - 1.0)
    v = (np.floor(y_now + now) - np.floor(y_prev + before)).astype(np.int64)
    inside = np.all(np.abs(v) <= V, axis=1)
    bins = np.zeros(len(v), dtype=np.int64)
    for ax in range(dim):
        bins += (v[:, ax] + V) * W ** ax
    counts = np.zeros(Q + 1, dtype=np.int64)
    counts[:Q] = np.bincount(bins[inside], minlength=Q)
    counts[Q] = int((~inside).sum())
    mom = [int(v[:, ax].sum()) for ax in range(dim)]
    for p in range(dim):
        for q in range(p, dim):
            mom.append(int((v[:, p] * v[:, q]).sum()))
    return counts, np.array(mom, dtype=np.int64)
