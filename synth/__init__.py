"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the method itself (no forces, no
integration, no binning): it only draws initial particle states, replica sizes
and hand-placed edge-case states from seeded numpy generators, so that both
sides of every parity test start from identical inputs.

Recipe (the paper's own MD input is not available; see the paper's section on
the two-dimensional Lennard-Jones gas for the shape it describes: a homogeneous
initial distribution with the kinetic energy of the target temperature):

* positions: a jittered grid.  With g = ceil(N^(1/d)) grid points per axis and
  spacing h = L/g, N distinct grid points are drawn at random and each is
  displaced uniformly by up to (h - r_min)/2 per axis, so that no two
  particles start closer than r_min (pure uniform sampling at these densities
  puts pairs at r << sigma, where single-precision LJ forces overflow);
* velocities: independent normal components with variance kT/m, centre-of-mass
  velocity removed, rescaled so that sum m v^2 / (d (N-1)) = kT exactly;
* both cast to float32, positions kept strictly inside [0, L).
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed):
    if isinstance(seed, np.random.Generator):
        return seed
    return np.random.default_rng(seed)


def lj_initial_state(dim, n, box, kT, seed, mass=1.0, r_min=0.8):
    """Return (pos, vel) as float32 arrays of shape (n, dim), pos in [0, box)."""
    rng = _rng(seed)
    box = float(box)
    g = int(math.ceil(n ** (1.0 / dim) - 1e-9))
    while g ** dim < n:
        g += 1
    h = box / g
    if h <= r_min:
        raise ValueError(f"density too high for a jittered grid: spacing {h} <= r_min {r_min}")
    pick = rng.permutation(g ** dim)[:n]
    grid = np.empty((n, dim), dtype=np.float64)
    for ax in range(dim):
        grid[:, ax] = (pick // (g ** ax)) % g
    jitter = (h - r_min) / 2.0
    pos = (grid + 0.5) * h + rng.uniform(-jitter, jitter, size=(n, dim))
    pos = np.mod(pos, box)
    pos32 = pos.astype(np.float32)
    top = np.nextafter(np.float32(box), np.float32(0.0))
    pos32 = np.where(pos32 >= np.float32(box), top, pos32)
    pos32 = np.where(pos32 < 0, np.float32(0.0), pos32).astype(np.float32)
    vel = maxwell_velocities(dim, n, kT, rng, mass=mass)
    return np.ascontiguousarray(pos32), vel


def maxwell_velocities(dim, n, kT, seed, mass=1.0):
    rng = _rng(seed)
    v = rng.normal(0.0, math.sqrt(kT / mass), size=(n, dim))
    if n > 1:
        v -= v.mean(axis=0, keepdims=True)
        s = float(np.sum(mass * v * v))
        if s > 0:
            v *= math.sqrt(kT * dim * (n - 1) / s)
    return np.ascontiguousarray(v.astype(np.float32))


def replica_sizes(n_replicas=512, seed=4, n_min=1024, n_max=65536, density=0.5, cell=4.0):
    """Replica sizes of the batched ensemble: N' log-uniform in [n_min, n_max]
    from SeedSequence(seed).spawn(n_replicas)[r]; each replica then gets
    M_r = round(sqrt(N'/density)/cell) lattice sites per axis and
    N_r = density * (cell M_r)^2 particles, so the density is exact and the box
    side cell*M_r is a whole number of lattice cells.  Returns (N_r, M_r)."""
    children = np.random.SeedSequence(seed).spawn(n_replicas)
    ns, ms = [], []
    for ch in children:
        r = np.random.default_rng(ch)
        nprime = math.exp(r.uniform(math.log(n_min), math.log(n_max)))
        m = max(3, int(round(math.sqrt(nprime / density) / cell)))
        ns.append(int(round(density * (cell * m) ** 2)))
        ms.append(m)
    return np.array(ns, dtype=np.int64), np.array(ms, dtype=np.int64)


def replica_seeds(n_replicas=512, seed=4):
    """Per-replica generators for the initial states of the ensemble."""
    return [np.random.default_rng(ch) for ch in
            np.random.SeedSequence(seed).spawn(n_replicas)]


def binning_edge_state(dim, M, k, vmax, n, seed, s):
    """Hand-placed edge cases for exact binning, in the cell/offset form.

    Returns a dict with int32 ``ucell`` (unwrapped MD-cell index per axis, i.e.
    wrapped cell + Mc * image), float32 ``off`` in [0, s), and the snapshot a
    lattice step earlier ``prev_ucell`` / ``prev_off``.  Mc = M * k MD cells per
    axis.  Offsets include 0 and the largest float32 below s; wrapped cells
    include 0 and Mc - 1; images include -2..2; lattice displacements include
    +-V (inside the window) and +-(V+1) (overflow)."""
    rng = _rng(seed)
    mc = M * k
    s32 = np.float32(s)
    top = np.nextafter(s32, np.float32(0.0))
    specials = np.array([0.0, top, s32 * np.float32(0.5), np.float32(1e-30),
                         np.nextafter(np.float32(0.0), np.float32(1.0))], dtype=np.float32)
    off = rng.uniform(0.0, float(s), size=(n, dim)).astype(np.float32)
    off = np.where(off >= s32, top, off)
    mask = rng.random(size=(n, dim)) < 0.4
    off = np.where(mask, specials[rng.integers(0, len(specials), size=(n, dim))], off)
    cell = rng.integers(0, mc, size=(n, dim))
    edge = rng.random(size=(n, dim)) < 0.3
    cell = np.where(edge, np.where(rng.random(size=(n, dim)) < 0.5, 0, mc - 1), cell)
    img = rng.integers(-2, 3, size=(n, dim))
    ucell = cell + mc * img
    # lattice displacement per axis, in lattice cells, then realised in MD cells
    choices = np.array([0, 1, -1, vmax, -vmax, vmax + 1, -(vmax + 1), 2, -2])
    vlat = choices[rng.integers(0, len(choices), size=(n, dim))]
    sub_now = np.floor_divide(ucell, k) * k
    prev_sub = rng.integers(0, k, size=(n, dim))
    prev_ucell = sub_now - vlat * k + prev_sub
    prev_off = rng.uniform(0.0, float(s), size=(n, dim)).astype(np.float32)
    prev_off = np.where(prev_off >= s32, top, prev_off)
    pmask = rng.random(size=(n, dim)) < 0.3
    prev_off = np.where(pmask, specials[rng.integers(0, len(specials), size=(n, dim))], prev_off)
    return {"ucell": ucell.astype(np.int32), "off": off.astype(np.float32),
            "prev_ucell": prev_ucell.astype(np.int32), "prev_off": prev_off.astype(np.float32)}
