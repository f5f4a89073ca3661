"""Parity of the binning on displaced and moving lattices (mdlg_get_shifts)
with the FP64 oracle, on identical positions: after every lattice step the
GPU state is read back and the oracle bins the same unwrapped positions on
every extra lattice; the integer counts and lattice moments must agree
exactly.  The unshifted extra lattice must reproduce the main histogram.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import make_system, say, unwrapped

pytestmark = pytest.mark.gpu

SHIFTS_2D = [[[0.0, 0.0], [0.0, 0.0]],          # the main lattice again
             [[0.25, 0.5], [0.0, 0.0]],         # displaced
             [[0.0, 0.0], [0.2, 0.0]],          # Galilean drift u = (0.2, 0)
             [[0.1, 0.3], [-0.35, 0.15]]]       # both


@pytest.mark.parametrize("dim,M,V,steps", [(2, 16, 3, 5), (3, 5, 1, 3)])
def test_shifted_lattices_match_oracle(dim, M, V, steps):
    from paper_1705_04368_amd import make_config
    say(f"shifted lattices dim={dim}")
    dx = 4.0
    n = 2048 if dim == 2 else 4740
    if dim == 2:
        shifts = np.array(SHIFTS_2D)
    else:
        shifts = np.array([[[0.0] * 3, [0.0] * 3], [[0.5, 0.25, 0.125], [0.3, -0.1, 0.05]]])
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=0.005, md_steps_per_lattice_step=40, vmax=V,
                      kT=1.0, shifts=shifts)
    pos, vel = synth.lj_initial_state(dim, n, M * dx, 1.0, seed=31 + dim)
    sysg = make_system(cfg, pos, vel)
    s = sysg.layout["cell_side"]
    lat = oracle.make_lattice(dim, (M,) * dim, dx, V)
    prev = unwrapped(sysg.get_state(), s)
    ref_c = np.zeros((len(shifts), sysg.Q + 1), np.int64)
    ref_m = np.zeros((len(shifts), dim + dim * (dim + 1) // 2), np.int64)
    for k in range(1, steps + 1):
        sysg.coarse_grain(1)
        now = unwrapped(sysg.get_state(), s)
        for j, (a, b) in enumerate(shifts):
            c, m = oracle.bin_shifted(lat, dim, prev, now, a, b, k)
            ref_c[j] += c
            ref_m[j] += m
        out = sysg.get_shifts()
        np.testing.assert_array_equal(out["counts"].astype(np.int64), ref_c)
        np.testing.assert_array_equal(out["moments"], ref_m)
        assert out["n_steps"] == k
        prev = now
    f = sysg.get_f()
    np.testing.assert_array_equal(out["counts"][0, :-1], f["counts"])
    assert int(out["counts"][0, -1]) == f["n_overflow"]


def test_shifted_lattices_batched_replicas():
    """A batch of two replicas on lattices of different sizes: every extra
    lattice bins each replica on that replica's own lattice; the counts and
    moments are the sums over the replicas."""
    from paper_1705_04368_amd import make_config
    say("shifted lattices, batched replicas")
    sizes, lats, dx, V, steps = (968, 2048), (11, 16), 4.0, 3, 4
    shifts = np.array(SHIFTS_2D)
    ps, vs = [], []
    for r, (n, m) in enumerate(zip(sizes, lats)):
        p, v = synth.lj_initial_state(2, n, m * dx, 1.0, seed=71 + r)
        ps.append(p)
        vs.append(v)
    cfg = make_config(2, list(sizes), [[m, m] for m in lats], lattice_dx=dx, dt=0.005,
                      md_steps_per_lattice_step=40, vmax=V, kT=1.0, shifts=shifts)
    sysg = make_system(cfg, np.concatenate(ps), np.concatenate(vs))
    s = sysg.layout["cell_side"]
    lat = [oracle.make_lattice(2, (m, m), dx, V) for m in lats]
    poff = np.concatenate([[0], np.cumsum(sizes)])
    prev = unwrapped(sysg.get_state(), s)
    ref_c = np.zeros((len(shifts), sysg.Q + 1), np.int64)
    ref_m = np.zeros((len(shifts), 5), np.int64)
    for k in range(1, steps + 1):
        sysg.coarse_grain(1)
        now = unwrapped(sysg.get_state(), s)
        for r in range(len(sizes)):
            sl = slice(poff[r], poff[r + 1])
            for j, (a, b) in enumerate(shifts):
                c, m = oracle.bin_shifted(lat[r], 2, prev[sl], now[sl], a, b, k)
                ref_c[j] += c
                ref_m[j] += m
        out = sysg.get_shifts()
        np.testing.assert_array_equal(out["counts"].astype(np.int64), ref_c)
        np.testing.assert_array_equal(out["moments"], ref_m)
        prev = now
    f = sysg.get_f()
    np.testing.assert_array_equal(out["counts"][0, :-1], f["counts"])


def test_shift_counter_restarts_with_the_accumulators():
    from paper_1705_04368_amd import make_config
    say("shift reset")
    dim, M, dx = 2, 16, 4.0
    shifts = np.array([[[0.0, 0.0], [0.3, 0.0]]])
    cfg = make_config(dim, 2048, M, lattice_dx=dx, dt=0.005, md_steps_per_lattice_step=20,
                      vmax=3, kT=1.0, shifts=shifts)
    pos, vel = synth.lj_initial_state(dim, 2048, M * dx, 1.0, seed=3)
    sysg = make_system(cfg, pos, vel)
    sysg.coarse_grain(3)
    sysg.reset_accumulators()
    assert sysg.get_shifts()["counts"].sum() == 0
    s = sysg.layout["cell_side"]
    lat = oracle.make_lattice(dim, (M,) * dim, dx, 3)
    prev = unwrapped(sysg.get_state(), s)
    sysg.coarse_grain(1)
    now = unwrapped(sysg.get_state(), s)
    c, m = oracle.bin_shifted(lat, dim, prev, now, shifts[0, 0], shifts[0, 1], 1)
    out = sysg.get_shifts()
    np.testing.assert_array_equal(out["counts"][0].astype(np.int64), c)
    np.testing.assert_array_equal(out["moments"][0], m)
