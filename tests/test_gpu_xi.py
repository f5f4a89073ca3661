"""Parity of the collision operator Xi_i(x,t) = n_i(x+v_i,t+1) - n_i(x,t)
(eq. Xi) recorded by the HIP path (mdlg_get_xi) with the FP64 oracle, on
identical positions: after every lattice step the GPU state is read back, the
oracle bins the same unwrapped positions (eq. MDni) and evaluates Xi; every
integer must agree exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import make_system, say, unwrapped

pytestmark = pytest.mark.gpu


def _run_and_compare(cfg, pos, vel, M, steps):
    dim = cfg.dim
    sysg = make_system(cfg, pos, vel)
    lay = sysg.layout
    s = lay["cell_side"]
    lat = oracle.make_lattice(dim, (M,) * dim, cfg.lattice_dx, cfg.vmax)
    Q = lay["n_velocities"]
    prev = unwrapped(sysg.get_state(), s)  # the snapshot the first lattice step bins against
    n_prev = None
    ref_sum = np.zeros((5, Q), np.int64)
    ref_site = np.zeros((lay["n_sites"], Q), np.int64)
    for t in range(1, steps + 1):
        sysg.coarse_grain(1)
        now = unwrapped(sysg.get_state(), s)
        n_now = oracle.bin_step(lat, dim, prev, now)["A"].astype(np.int64)
        out = sysg.get_xi(per_site=True, last=True)
        if n_prev is not None:
            xi = oracle.collision_operator(lat, dim, n_prev, n_now)
            np.testing.assert_array_equal(out["xi_last"], xi)
            ref_site += xi
            ref_sum += np.stack([xi.sum(0), (xi * xi).sum(0), (xi * n_prev).sum(0),
                                 n_prev.sum(0), (n_prev * n_prev).sum(0)])
        np.testing.assert_array_equal(np.stack([out[k] for k in ("xi", "xi2", "xi_n", "n", "n2")]),
                                      ref_sum)
        np.testing.assert_array_equal(out["xi_site"], ref_site)
        assert out["n_steps"] == t - 1
        prev, n_prev = now, n_now
    return sysg, ref_sum


def test_xi_single_particle():
    from paper_1705_04368_amd import make_config
    say("xi single particle")
    cfg = make_config(2, 1, 4, lattice_dx=4.0, dt=0.25, md_steps_per_lattice_step=4, vmax=1,
                      forces_off=True, md_cell_split=1, sort_every=1, collision_stats=True)
    pos = np.array([[1.1 * 4.0, 1.5 * 4.0]], np.float32)
    vel = np.array([[4.0 / 3.0, 0.0]], np.float32)
    _, sums = _run_and_compare(cfg, pos, vel, 4, 6)
    assert np.abs(sums[0]).sum() > 0  # the particle changed lattice velocity


@pytest.mark.parametrize("dim,M,V", [(2, 16, 3), (3, 5, 1)])
def test_xi_lj_gas(dim, M, V):
    from paper_1705_04368_amd import make_config
    say(f"xi LJ gas dim={dim}")
    dx = 4.0
    n = 2048 if dim == 2 else 4740
    # Delta t long enough for sub-cell moves to cross cells often
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=0.005, md_steps_per_lattice_step=40, vmax=V,
                      kT=1.0, collision_stats=True)
    pos, vel = synth.lj_initial_state(dim, n, M * dx, 1.0, seed=21 + dim)
    sysg, sums = _run_and_compare(cfg, pos, vel, M, 5)
    # mass conservation (eq. Mom0): no displacement left the window
    f = sysg.get_f()
    assert f["n_overflow"] == 0
    out = sysg.get_xi(last=True)
    np.testing.assert_array_equal(out["xi_last"].sum(axis=1), 0)
    assert int(sums[0].sum()) == 0


def test_xi_chain_restarts_after_md_steps():
    from paper_1705_04368_amd import make_config
    say("xi chain restart")
    cfg = make_config(2, 2048, 16, lattice_dx=4.0, dt=0.005, md_steps_per_lattice_step=20,
                      vmax=3, kT=1.0, collision_stats=True)
    pos, vel = synth.lj_initial_state(2, 2048, 64.0, 1.0, seed=5)
    sysg = make_system(cfg, pos, vel)
    sysg.coarse_grain(3)
    assert sysg.get_xi()["n_steps"] == 2
    sysg.step(7)  # plain MD: the next lattice step starts a new chain
    sysg.coarse_grain(2)
    assert sysg.get_xi()["n_steps"] == 3
    sysg.reset_accumulators()
    assert sysg.get_xi()["n_steps"] == 0


def test_xi_batched_replicas():
    """Two replicas of different lattices in one batch: each replica's Xi
    wraps on its own lattice (x + v_i taken modulo that replica's sites);
    the per-site fields are the replicas' fields one after the other and the
    moments their sums."""
    from paper_1705_04368_amd import make_config
    say("xi batched replicas")
    sizes, lats, dx = (968, 2048), (11, 16), 4.0
    ps, vs = [], []
    for r, (n, m) in enumerate(zip(sizes, lats)):
        p, v = synth.lj_initial_state(2, n, m * dx, 1.0, seed=61 + r)
        ps.append(p)
        vs.append(v)
    cfg = make_config(2, list(sizes), [[m, m] for m in lats], lattice_dx=dx, dt=0.005,
                      md_steps_per_lattice_step=40, vmax=3, kT=1.0, collision_stats=True)
    sysg = make_system(cfg, np.concatenate(ps), np.concatenate(vs))
    s = sysg.layout["cell_side"]
    Q = sysg.layout["n_velocities"]
    lat = [oracle.make_lattice(2, (m, m), dx, 3) for m in lats]
    poff = np.concatenate([[0], np.cumsum(sizes)])
    prev = unwrapped(sysg.get_state(), s)
    n_prev = None
    ref_sum = np.zeros((5, Q), np.int64)
    ref_site = np.zeros((sum(m * m for m in lats), Q), np.int64)
    for t in range(1, 5):
        sysg.coarse_grain(1)
        now = unwrapped(sysg.get_state(), s)
        n_now = [oracle.bin_step(lat[r], 2, prev[poff[r]:poff[r + 1]],
                                 now[poff[r]:poff[r + 1]])["A"].astype(np.int64)
                 for r in range(len(sizes))]
        out = sysg.get_xi(per_site=True, last=True)
        if n_prev is not None:
            xi = [oracle.collision_operator(lat[r], 2, n_prev[r], n_now[r]) for r in range(len(sizes))]
            np.testing.assert_array_equal(out["xi_last"], np.concatenate(xi))
            ref_site += np.concatenate(xi)
            for r in range(len(sizes)):
                ref_sum += np.stack([xi[r].sum(0), (xi[r] * xi[r]).sum(0), (xi[r] * n_prev[r]).sum(0),
                                     n_prev[r].sum(0), (n_prev[r] * n_prev[r]).sum(0)])
        np.testing.assert_array_equal(np.stack([out[k] for k in ("xi", "xi2", "xi_n", "n", "n2")]),
                                      ref_sum)
        np.testing.assert_array_equal(out["xi_site"], ref_site)
        assert out["n_steps"] == t - 1
        prev, n_prev = now, n_now
    assert np.abs(ref_sum[0]).sum() > 0
