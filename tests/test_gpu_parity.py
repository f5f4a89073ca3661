"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (per particle / per site):
* binning and all integer accumulators: bit-exact on identical positions;
* forces: |F_gpu - F_ref| <= 1e-5 max(|F_ref|, F_rms), F_ref the FP64 oracle
  on the same float32 positions;
* 20-step trajectories from one state: |x_gpu - x_ref| <= 1e-4 sigma
  (unwrapped) and |v_gpu - v_ref| <= 1e-4 sqrt(kT/m);
* ideal gas: identical counts up to particles within float rounding of a
  cell edge, and the wedge / closed form of the paper within sampling error.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import closed_form as cf
from tests.gpu_util import force_error, make_system, say, unwrapped, wrapped

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ binning

@pytest.mark.parametrize("dim,M,k,vmax", [(2, 8, 1, 3), (2, 6, 2, 1), (2, 5, 4, 0),
                                         (3, 4, 1, 2), (3, 3, 2, 1)])
def test_binning_bit_exact_edge_cases(dim, M, k, vmax):
    from paper_1705_04368_amd import make_config
    dx = 4.0
    n = 3000 if dim == 2 else 4000
    say(f"binning edge cases dim={dim} M={M} k={k} V={vmax}")
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=0.005, md_steps_per_lattice_step=1, vmax=vmax,
                      forces_off=True, md_cell_split=k, sort_every=1)
    pos, _ = synth.lj_initial_state(dim, n, M * dx, 1.0, seed=5, r_min=0.0)
    sysg = make_system(cfg, pos, np.zeros_like(pos))
    s = sysg.layout["cell_side"]
    assert sysg.layout["md_cell_split"] == k
    st = synth.binning_edge_state(dim, M, k, vmax, n, seed=17 + dim + k, s=s)
    sysg.set_state(st["ucell"], st["off"], np.zeros((n, dim), np.float32),
                   st["prev_ucell"], st["prev_off"])
    sysg.coarse_grain(1)
    out = sysg.get_f(per_site=True)
    xu_now = st["ucell"].astype(np.float64) * s + st["off"].astype(np.float64)
    xu_prev = st["prev_ucell"].astype(np.float64) * s + st["prev_off"].astype(np.float64)
    lat = oracle.make_lattice(dim, (M,) * dim, dx, vmax)
    ref = oracle.bin_step(lat, dim, xu_prev, xu_now)
    got_A = np.rint(out["f_site"]).astype(np.int64)
    got_m = np.rint(out["mom_site"]).astype(np.int64)
    np.testing.assert_array_equal(got_A, ref["A"].astype(np.int64))
    np.testing.assert_array_equal(got_m, ref["mom"])
    assert out["n_overflow"] == int(ref["mom"][:, 1].sum()) > 0
    np.testing.assert_array_equal(out["counts"], ref["A"].sum(axis=0))
    np.testing.assert_allclose(out["disp_sum"], ref["dsum"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(out["disp_sq"], ref["dsq"], rtol=1e-12, atol=1e-9)
    # the snapshot moved to the current positions
    after = sysg.get_state()
    np.testing.assert_array_equal(after["prev_ucell"], st["ucell"])
    np.testing.assert_array_equal(after["ucell"], st["ucell"])
    np.testing.assert_allclose(after["prev_off"], st["off"], rtol=0, atol=1e-37)


# ------------------------------------------------------------------ forces

def _force_case(dim, seed, k, brick=(0, 0, 0), dense=False, equil_steps=0):
    from paper_1705_04368_amd import make_config
    if dim == 2:
        # dense: rho = 1.13, so a 64x3-cell brick stages more particles than one
        # LDS chunk holds and the kernel streams its halo in several chunks
        M, n, dx = (16, 2048, 4.0) if not dense else (40, 28877, 4.0)
    else:
        M, n, dx = 5, 4740, 4.0
    box = M * dx
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=seed, r_min=0.8 if not dense else 0.82)
    if equil_steps:
        md = oracle.make_md(dim, n, box, dt=0.005)
        ost = oracle.OracleState(md, pos, vel)
        ost.run(equil_steps, thermo_every=10, kT=1.0)
        pos = ost.x.astype(np.float32)
        pos = np.where(pos >= np.float32(box), np.float32(0.0), pos)
        vel = ost.v.astype(np.float32)
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=0.005, vmax=1 if dim == 3 else 3,
                      md_cell_split=k, brick=brick, kT=1.0)
    return cfg, pos, vel, box, n, M


@pytest.mark.parametrize("dim,k,brick,dense,equil", [
    (2, 1, (0, 0, 0), False, 0), (2, 2, (0, 0, 0), False, 0), (2, 4, (0, 0, 0), False, 0),
    (2, 1, (64, 3, 1), True, 0), (2, 1, (5, 2, 1), False, 300), (3, 1, (0, 0, 0), False, 0),
    (3, 2, (0, 0, 0), False, 0), (3, 2, (3, 2, 2), False, 0)])
def test_forces_match_oracle(dim, k, brick, dense, equil):
    cfg, pos, vel, box, n, M = _force_case(dim, 31 + k, k, brick, dense, equil)
    say(f"forces dim={dim} k={k} brick={brick} dense={dense} equil={equil}")
    sysg = make_system(cfg, pos, vel)
    st = sysg.get_state()
    s = sysg.layout["cell_side"]
    mc = M * sysg.layout["md_cell_split"]
    xw = wrapped(st, s, mc)
    # the state the GPU holds is exactly the input (float32 -> cell + offset)
    np.testing.assert_array_equal(xw, pos.astype(np.float64))
    md = oracle.make_md(dim, n, box)
    acc, _ = oracle.forces(md, xw)
    err = force_error(st["acc"], acc)
    say(f"  max rel force error {err.max():.3e}  median {np.median(err):.3e}")
    assert err.max() <= 1e-5
    np.testing.assert_array_equal(st["vel"], vel)


# ------------------------------------------------------------------ trajectories

@pytest.mark.parametrize("dim,sort_every", [(2, 0), (2, 1), (2, 7), (3, 0)])
def test_twenty_step_trajectory(dim, sort_every):
    # from an equilibrated state (oracle, 300 thermostatted steps)
    cfg, pos, vel, box, n, M = _force_case(dim, 77, 2 if dim == 3 else 1, equil_steps=300)
    cfg.sort_every = sort_every
    say(f"trajectory dim={dim} sort_every={sort_every}")
    sysg = make_system(cfg, pos, vel)
    sysg.step(20)
    st = sysg.get_state()
    md = oracle.make_md(dim, n, box, dt=0.005)
    ost = oracle.OracleState(md, pos, vel)
    ost.run(20)
    dxmax = np.abs(unwrapped(st, sysg.layout["cell_side"]) - ost.unwrapped).max()
    dvmax = np.abs(st["vel"].astype(np.float64) - ost.v).max()
    say(f"  max |dx| {dxmax:.3e}  max |dv| {dvmax:.3e}")
    assert dxmax <= 1e-4
    assert dvmax <= 1e-4


# ------------------------------------------------------------------ ideal gas

def test_ideal_gas_counts_match_oracle_and_closed_form():
    from paper_1705_04368_amd import make_config
    dim, n, M, dx, kT = 2, 2048, 16, 4.0, 1.0
    box = M * dx
    pos, vel = synth.lj_initial_state(dim, n, box, kT, seed=1)
    steps, T = 320, 40  # Delta t = 1.6: a = 0.4
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=0.005, md_steps_per_lattice_step=steps, vmax=3,
                      forces_off=True, kT=kT)
    say("ideal gas f_i")
    sysg = make_system(cfg, pos, vel)
    sysg.coarse_grain(T)
    g = sysg.get_f(per_site=True)
    md = oracle.make_md(dim, n, box, dt=0.005, forces_off=True)
    ost = oracle.OracleState(md, pos, vel, use_cells=False)
    lat = oracle.make_lattice(dim, (M, M), dx, 3)
    o = ost.mdlg(lat, steps, T)
    go = g["counts"].astype(np.int64)
    oo = o["A"].sum(axis=0).astype(np.int64)
    # Free flight has the closed form x0 + v t.  The float32 cell offsets drift
    # from it by eps (measured at the end); a particle can bin differently only
    # at a lattice step where its exact position lies within eps of a cell
    # edge, and each such event moves one count between two bins.
    st = sysg.get_state()
    s = sysg.layout["cell_side"]
    x0 = pos.astype(np.float64)
    v = vel.astype(np.float64)
    dt_lat = steps * 0.005
    eps = np.abs(unwrapped(st, s) - (x0 + v * dt_lat * T)).max()
    near = 0
    for t in range(T + 1):
        y = (x0 + v * dt_lat * t) / dx
        near += int((np.abs(y - np.rint(y)) * dx < eps).any(axis=1).sum())
    say(f"  drift eps {eps:.2e}, near-edge events {near}, count mismatch {np.abs(go - oo).sum()}")
    assert eps < 5e-3
    assert np.abs(go - oo).sum() <= 2 * near, (go, oo)
    f_meas = g["f"] / (n / M ** 2)
    f_cf = cf.feq_over_rho(dim, 3, 0.4)
    big = f_cf > 1e-3
    np.testing.assert_allclose(f_meas[big], f_cf[big], rtol=0.08)
    msd = g["disp_sq"] / (n * T)
    np.testing.assert_allclose(msd, kT * 1.6 ** 2, rtol=0.08)


# ------------------------------------------------------------------ graph / eager, replicas

def _run_forces_off(env_graph, n_rep_sizes, lattices, T=6):
    from paper_1705_04368_amd import make_config
    old = os.environ.get("MDLG_NO_GRAPH")
    os.environ["MDLG_NO_GRAPH"] = "0" if env_graph else "1"
    try:
        dim = 2
        pos_all, vel_all = [], []
        for r, (n, m) in enumerate(zip(n_rep_sizes, lattices)):
            p, v = synth.lj_initial_state(dim, n, 4.0 * m, 1.0, seed=100 + r)
            pos_all.append(p)
            vel_all.append(v)
        cfg = make_config(dim, n_rep_sizes, [[m, m] for m in lattices], lattice_dx=4.0, dt=0.01,
                          md_steps_per_lattice_step=30, vmax=2, forces_off=True, kT=1.0,
                          sort_every=4)
        sysg = make_system(cfg, np.concatenate(pos_all), np.concatenate(vel_all))
        sysg.coarse_grain(T)
        return sysg.get_f(per_site=True), sysg.get_state()
    finally:
        if old is None:
            os.environ.pop("MDLG_NO_GRAPH", None)
        else:
            os.environ["MDLG_NO_GRAPH"] = old


def test_graph_replay_equals_eager_bitwise():
    say("graph vs eager")
    a, sa = _run_forces_off(True, [1500], [14])
    b, sb = _run_forces_off(False, [1500], [14])
    np.testing.assert_array_equal(a["f_site"], b["f_site"])
    np.testing.assert_array_equal(a["mom_site"], b["mom_site"])
    for key in ("ucell", "off", "vel", "prev_ucell", "prev_off"):
        np.testing.assert_array_equal(sa[key], sb[key])


def _run_long_steps(env_graph, steps, T=3):
    from paper_1705_04368_amd import make_config
    old = os.environ.get("MDLG_NO_GRAPH")
    os.environ["MDLG_NO_GRAPH"] = "0" if env_graph else "1"
    try:
        n, M = 2048, 16
        pos, vel = synth.lj_initial_state(2, n, 4.0 * M, 1.0, seed=61)
        sh = np.zeros((2, 2, 2))
        sh[1, 1, 0] = 0.25
        # free flight: the sequencing is under test (forces on:
        # test_gpu_determinism)
        cfg = make_config(2, n, M, lattice_dx=4.0, dt=0.004, md_steps_per_lattice_step=steps, vmax=3,
                          kT=1.0, sort_every=7, collision_stats=True, shifts=sh, forces_off=True)
        sysg = make_system(cfg, pos, vel)
        sysg.coarse_grain(T)
        return (sysg.get_f(per_site=True), sysg.get_state(), sysg.get_xi(per_site=True, last=True),
                sysg.get_shifts())
    finally:
        if old is None:
            os.environ.pop("MDLG_NO_GRAPH", None)
        else:
            os.environ["MDLG_NO_GRAPH"] = old


def test_long_lattice_steps_replay_in_blocks():
    # 450 MD steps per lattice step: replayed as graphs of whole rebuild
    # intervals (196 steps) and a tail with the binning; bitwise the same as
    # eager launches, with the collision operator and a drifting lattice on
    # (free flight: the sequencing is under test, not the forces)
    say("long lattice steps: block graphs vs eager")
    a = _run_long_steps(True, 450)
    b = _run_long_steps(False, 450)
    np.testing.assert_array_equal(a[0]["f_site"], b[0]["f_site"])
    np.testing.assert_array_equal(a[0]["mom_site"], b[0]["mom_site"])
    assert a[0]["n_lattice_steps"] == b[0]["n_lattice_steps"] == 3
    for key in ("ucell", "off", "vel", "prev_ucell", "prev_off"):
        np.testing.assert_array_equal(a[1][key], b[1][key])
    for key in ("xi", "xi2", "xi_n", "xi_site", "xi_last"):
        np.testing.assert_array_equal(a[2][key], b[2][key])
    assert a[2]["n_steps"] == b[2]["n_steps"] == 2
    for key in ("counts", "moments", "n_steps"):
        np.testing.assert_array_equal(np.asarray(a[3][key]), np.asarray(b[3][key]))
    assert a[3]["n_steps"] == 3


def test_batched_replicas_equal_separate_runs():
    sizes, lats = [968, 2048, 1500], [11, 16, 14]
    say("batched replicas vs separate")
    both, sboth = _run_forces_off(True, sizes, lats)
    off_site, off_part = 0, 0
    for r, (n, m) in enumerate(zip(sizes, lats)):
        p, v = synth.lj_initial_state(2, n, 4.0 * m, 1.0, seed=100 + r)
        from paper_1705_04368_amd import make_config
        cfg = make_config(2, [n], [[m, m]], lattice_dx=4.0, dt=0.01, md_steps_per_lattice_step=30,
                          vmax=2, forces_off=True, kT=1.0, sort_every=4)
        single = make_system(cfg, p, v)
        single.coarse_grain(6)
        fs = single.get_f(per_site=True)
        ns = m * m
        np.testing.assert_array_equal(both["f_site"][off_site:off_site + ns], fs["f_site"])
        np.testing.assert_array_equal(both["mom_site"][off_site:off_site + ns], fs["mom_site"])
        ss = single.get_state()
        np.testing.assert_array_equal(sboth["off"][off_part:off_part + n], ss["off"])
        off_site += ns
        off_part += n


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_replica_forces_match_oracle(dim):
    from paper_1705_04368_amd import make_config
    if dim == 2:
        sizes, lats, kT = [968, 2048, 1250], [11, 16, 10], 1.0
    else:
        # rho = 0.593 on lattices of 4, 5 and 6 cells of 4 sigma
        sizes, lats, kT = [2429, 4744, 8198], [4, 5, 6], 1.5
    pos_all, vel_all = [], []
    for r, (n, m) in enumerate(zip(sizes, lats)):
        p, v = synth.lj_initial_state(dim, n, 4.0 * m, kT, seed=300 + r)
        pos_all.append(p)
        vel_all.append(v)
    say(f"replica forces, {dim}D")
    cfg = make_config(dim, sizes, [[m] * dim for m in lats], lattice_dx=4.0,
                      dt=0.005 if dim == 2 else 0.004, vmax=3 if dim == 2 else 2, kT=kT)
    sysg = make_system(cfg, np.concatenate(pos_all), np.concatenate(vel_all))
    st = sysg.get_state()
    s = sysg.layout["cell_side"]
    k = sysg.layout["md_cell_split"]
    off = 0
    for r, (n, m) in enumerate(zip(sizes, lats)):
        sl = slice(off, off + n)
        sub = {key: val[sl] for key, val in st.items()}
        xw = wrapped(sub, s, m * k)
        np.testing.assert_array_equal(xw, pos_all[r].astype(np.float64))
        acc, _ = oracle.forces(oracle.make_md(dim, n, 4.0 * m), xw)
        assert force_error(sub["acc"], acc).max() <= 1e-5
        off += n


# ------------------------------------------------------------------ state I/O, errors

def test_state_roundtrip_and_readout_does_not_perturb():
    cfg, pos, vel, box, n, M = _force_case(2, 5, 1)
    say("state round trip")
    a = make_system(cfg, pos, vel)
    a.step(10)
    mid = a.get_state()
    a.step(10)
    sa = a.get_state()
    b = make_system(cfg, pos, vel)
    b.step(20)
    sb = b.get_state()
    s = a.layout["cell_side"]
    # a readout completes the half kick and the next step starts from it:
    # bit for bit the same trajectory (the slots, hence the sums, are fixed)
    np.testing.assert_array_equal(unwrapped(sa, s), unwrapped(sb, s))
    np.testing.assert_array_equal(sa["vel"], sb["vel"])
    c = make_system(cfg, pos, vel)
    c.set_state(mid["ucell"], mid["off"], mid["vel"], mid["prev_ucell"], mid["prev_off"])
    sc = c.get_state()
    for key in ("ucell", "off", "vel", "prev_ucell", "prev_off"):
        np.testing.assert_array_equal(sc[key], mid[key])


def test_unstable_step_is_reported():
    from paper_1705_04368_amd import MdlgError
    cfg, pos, vel, box, n, M = _force_case(2, 9, 1)
    cfg.sort_every = 10
    vel = vel.copy()
    vel[0] = [400.0, 0.0]  # 2 sigma per step: past the stencil's reach within a few
    say("unstable step")
    sysg = make_system(cfg, pos, vel)
    sysg.step(3)
    with pytest.raises(MdlgError) as e:
        sysg.sync()
    assert e.value.status == -4


def test_force_launches_stop_after_an_error():
    """Once the device error word is set (every error is fatal), force launches
    do nothing: the fast particle keeps the lists stale, so each launch that
    still ran would walk the cells and count a fallback; none is counted after
    the error."""
    import ctypes as C

    from paper_1705_04368_amd.native import load
    cfg, pos, vel, box, n, M = _force_case(2, 9, 1)
    cfg.sort_every = 10
    vel = vel.copy()
    vel[0] = [400.0, 0.0]  # past the speed cap at once, past the reach within a step or two
    say("force launches after an error")
    sysg = make_system(cfg, pos, vel)
    assert sysg.layout["pair_slots"] > 0
    sysg.step(3)
    lib = load()
    f1, f2 = C.c_int64(-1), C.c_int64(-1)
    assert lib.mdlg_get_list_fallbacks(sysg.handle, C.byref(f1)) == -4
    sysg.step(50)
    assert lib.mdlg_get_list_fallbacks(sysg.handle, C.byref(f2)) == -4
    assert 0 <= f1.value <= 3
    assert f2.value == f1.value


def test_empty_lattice_steps_and_single_particle():
    from paper_1705_04368_amd import make_config
    say("single particle")
    cfg = make_config(2, 1, 4, lattice_dx=4.0, dt=0.25, md_steps_per_lattice_step=4, vmax=1,
                      forces_off=True, md_cell_split=1, sort_every=1)
    # the worked example of the one-dimensional thought experiment, scaled to
    # 4-sigma cells: start 1.1 cells in, move 1/3 cell per lattice time step
    pos = np.array([[1.1 * 4.0, 1.5 * 4.0]], np.float32)
    vel = np.array([[4.0 / 3.0, 0.0]], np.float32)
    sysg = make_system(cfg, pos, vel)
    sysg.coarse_grain(0)
    hist = []
    for t in range(6):
        before = sysg.get_f(per_site=True)["f_site"] * max(t, 1)
        sysg.coarse_grain(1)
        after = sysg.get_f(per_site=True)["f_site"] * (t + 1)
        hist.append(np.rint(after - (before if t else 0)).astype(np.int64))
    f0, f1 = 4, 5  # bins of v = (0, 0) and v = (+1, 0) for V = 1
    expected = [(1, f0), (1, f0), (2, f1), (2, f0), (2, f0), (3, f1)]
    for t, (x, b) in enumerate(expected):
        site = x + 4 * 1
        nz = np.argwhere(hist[t] > 0)
        assert nz.tolist() == [[site, b]], (t, nz)


# ------------------------------------------------------------------ pair lists

@pytest.mark.parametrize("dim", [2, 3])
def test_pair_lists_match_cell_walk_and_oracle(dim):
    # the same 40 MD steps with per-particle pair lists (rebuilt with the cell
    # list every 8 steps) and with the cell walk at every step, in the same
    # layout: both sum the pairs within r_cut in the order of the brick's
    # staging (list entries beyond r_cut add exact zeros), so the runs agree
    # bit for bit; both within the bars of the oracle
    cfg_l, pos, vel, box, n, M = _force_case(dim, 78, 2 if dim == 3 else 1, equil_steps=300)
    cfg_c, *_ = _force_case(dim, 78, 2 if dim == 3 else 1)
    say(f"pair lists vs cell walk dim={dim}")
    sl = make_system(cfg_l, pos, vel)
    lay = sl.layout
    for c in (cfg_l, cfg_c):
        c.sort_every = 8
        c.md_cell_split = lay["md_cell_split"]
        c.brick_x, c.brick_y, c.brick_z = lay["brick"]
        c.block_threads = lay["block_threads"]
    cfg_c.no_pair_list = 1
    sl = make_system(cfg_l, pos, vel)
    sc = make_system(cfg_c, pos, vel)
    assert sl.layout["pair_slots"] > 0 and sc.layout["pair_slots"] == 0
    s = sl.layout["cell_side"]
    f_l, f_c = sl.get_state()["acc"], sc.get_state()["acc"]
    np.testing.assert_array_equal(f_l, f_c)
    md = oracle.make_md(dim, n, box, dt=0.005)
    acc, _ = oracle.forces(md, wrapped(sl.get_state(), s, M * sl.layout["md_cell_split"]))
    assert force_error(f_l, acc).max() <= 1e-5
    sl.step(40)
    sc.step(40)
    a, b = sl.get_state(), sc.get_state()
    for key in ("ucell", "off", "vel", "acc"):
        np.testing.assert_array_equal(a[key], b[key])
    ost = oracle.OracleState(md, pos, vel)
    ost.run(40)
    assert np.abs(unwrapped(a, s) - ost.unwrapped).max() <= 1e-4
    assert np.abs(a["vel"].astype(np.float64) - ost.v).max() <= 1e-4


def test_pair_list_overflow_falls_back_to_cell_walk():
    # all particles packed into a sixteenth of the box: lists in the packed
    # region hold about sixteen times the neighbours the mean density
    # predicts, more than the slots, so those bricks walk their cells (one-cell
    # bricks, so that their halo still fits one LDS chunk)
    from paper_1705_04368_amd import make_config
    M, dx, n = 16, 4.0, 256
    box = M * dx
    pos, vel = synth.lj_initial_state(2, n, box / 4, 1.0, seed=12, r_min=0.8)
    cfg = make_config(2, n, M, lattice_dx=dx, dt=0.005, vmax=3, md_cell_split=1, kT=1.0,
                      brick=(1, 1, 1))
    say("pair-list overflow")
    sysg = make_system(cfg, pos, vel)
    kmax = sysg.layout["pair_slots"]
    s = sysg.layout["cell_side"]
    st = sysg.get_state()
    md = oracle.make_md(2, n, box)
    xw = wrapped(st, s, M)
    acc, _ = oracle.forces(md, xw)
    assert force_error(st["acc"], acc).max() <= 1e-5
    # the packed region really exceeds the slots
    d = xw[:, None, :] - xw[None, :, :]
    d -= box * np.rint(d / box)
    r = np.sqrt((d ** 2).sum(-1))
    rl = 2.5 + 2 * sysg.layout["skin"]
    assert ((r < rl).sum(1) - 1).max() > kmax


def test_stale_pair_lists_walk_the_cells():
    # two particles far apart; one moves 0.15 sigma per step inside its cell,
    # so the displacement bound passes the lists' skin after a few steps: the
    # rest of the interval walks the cells (counted), with no error, and the
    # flight stays exact
    from paper_1705_04368_amd import make_config
    cfg = make_config(2, 2, 4, lattice_dx=4.0, dt=0.005, vmax=1, md_cell_split=1, kT=1.0,
                      sort_every=18)
    pos = np.array([[1.0, 2.0], [9.0, 10.0]], np.float32)
    vel = np.array([[30.0, 0.0], [0.0, 0.0]], np.float32)
    say("stale pair lists: cell walk")
    sysg = make_system(cfg, pos, vel)
    m = sysg.layout["skin"]
    assert sysg.layout["pair_slots"] > 0 and sysg.layout["sort_every"] == 18
    steps = int(np.ceil(m / (30.0 * 0.005))) + 2
    assert 1.0 + 30.0 * 0.005 * steps < 4.0  # still inside its cell
    sysg.step(steps)
    sysg.sync()
    assert sysg.list_fallbacks() >= 1
    x = unwrapped(sysg.get_state(), sysg.layout["cell_side"])
    assert abs(x[0, 0] - (1.0 + 30.0 * 0.005 * steps)) < 1e-4
    assert abs(x[1, 0] - 9.0) < 1e-6


@pytest.mark.parametrize("speed,stale", [(6.0, True), (2.0, False)])
def test_displacement_bound_sums_the_drifts(speed, stale):
    # one particle at a speed under the cap 8 (kT/m)^(1/2), so that only the
    # bound summed over the drifts since the build (carried from launch to
    # launch) can mark the lists stale: at 6 sigma/tau it passes the skin
    # inside the 18-step interval and the later launches walk the cells; at
    # 2 sigma/tau it never does.  The flight is exact either way.
    from paper_1705_04368_amd import make_config
    cfg = make_config(2, 2, 4, lattice_dx=4.0, dt=0.005, vmax=1, md_cell_split=1, kT=1.0,
                      sort_every=18)
    pos = np.array([[1.0, 2.0], [9.0, 10.0]], np.float32)
    vel = np.array([[speed, 0.0], [0.0, 0.0]], np.float32)
    say(f"displacement bound, speed {speed}")
    sysg = make_system(cfg, pos, vel)
    skin = sysg.layout["skin"]
    assert sysg.layout["pair_slots"] > 0 and sysg.layout["sort_every"] == 18
    cap = 8.0 * 0.005  # one drift at the speed cap
    assert speed < 8.0
    # the bound before drift n is about n speed dt + cap: past the skin at
    # 6 sigma/tau by drift 10, below it at 2 sigma/tau through drift 17
    if stale:
        assert 10 * speed * 0.005 + cap > skin * 1.01
    else:
        assert 17 * speed * 0.005 + cap < skin * 0.99
    sysg.step(18)
    sysg.sync()
    fb = sysg.list_fallbacks()
    say(f"  skin {skin:.4f}, launches that walked the cells: {fb}")
    if stale:
        assert 1 <= fb <= 9
    else:
        assert fb == 0
    x = unwrapped(sysg.get_state(), sysg.layout["cell_side"])
    assert abs(x[0, 0] - (1.0 + speed * 0.005 * 18)) < 1e-4
    assert abs(x[1, 0] - 9.0) < 1e-6


@pytest.mark.parametrize("dim,lists", [(2, True), (2, False), (3, True)])
def test_particles_past_the_margin_stay_exact(dim, lists):
    # The rebuild margin is sized for kT = 0.01 while the particles move at
    # kT = 1, so between rebuilds many leave their cells by more than the
    # margin, none by the stencil's reach.  Speeds above the cap mark the
    # lists stale at the first drift; the cell walk, pruned with the reach,
    # then follows the oracle over two rebuild intervals with no error.
    cfg, pos, vel, box, n, M = _force_case(dim, 77, 2 if dim == 3 else 1, equil_steps=300)
    cfg.kT = 0.01
    cfg.sort_every = 18
    cfg.no_pair_list = 0 if lists else 1
    say(f"past the margin dim={dim} lists={lists}")
    sysg = make_system(cfg, pos, vel)
    lay = sysg.layout
    s, margin, reach = lay["cell_side"], lay["margin"], lay["reach"]
    assert lay["sort_every"] == 18 and (lay["pair_slots"] > 0) == lists
    md = oracle.make_md(dim, n, box, dt=0.005)
    ost = oracle.OracleState(md, pos, vel)
    # largest excursion outside the cell of the last rebuild (steps 0 and
    # 18), over the drifts that no rebuild follows
    excursion = 0.0
    cell = np.floor(ost.unwrapped / s)
    for step in range(1, 37):
        ost.run(1)
        x = ost.unwrapped
        if step % 18:
            out = np.maximum(cell * s - x, x - (cell + 1) * s)
            excursion = max(excursion, float(out.max()))
        else:
            cell = np.floor(x / s)
    say(f"  margin {margin:.4f}, reach {reach:.4f}, largest excursion {excursion:.4f}")
    assert margin < excursion < reach
    sysg.step(36)
    sysg.sync()
    if lists:
        assert sysg.list_fallbacks() >= 1
    st = sysg.get_state()
    dxmax = np.abs(unwrapped(st, s) - ost.unwrapped).max()
    dvmax = np.abs(st["vel"].astype(np.float64) - ost.v).max()
    say(f"  max |dx| {dxmax:.3e}  max |dv| {dvmax:.3e}")
    assert dxmax <= 1e-4
    assert dvmax <= 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_forces_at_every_step_between_rebuilds(dim):
    # Forces at each MD step of one rebuild interval (the pair lists, built
    # at its start, age by one step each time) against the oracle on the
    # GPU's own positions, with a few particles sent off at 7 (kT/m)^(1/2) so
    # that the largest displacement since the build grows past half the
    # lists' skin inside the interval.
    from tests.gpu_util import check_forces_at_cutoff
    cfg, pos, vel, box, n, M = _force_case(dim, 91, 2 if dim == 3 else 1, equil_steps=300)
    cfg.sort_every = 12
    rng = np.random.default_rng(5)
    hot = rng.choice(n, size=8, replace=False)
    d = rng.normal(size=(8, dim))
    vel = vel.copy()
    vel[hot] = (7.0 * d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    say(f"forces between rebuilds dim={dim}")
    sysg = make_system(cfg, pos, vel)
    m = sysg.layout["skin"]
    s = sysg.layout["cell_side"]
    mc = M * sysg.layout["md_cell_split"]
    assert sysg.layout["pair_slots"] > 0 and sysg.layout["sort_every"] == 12
    md = oracle.make_md(dim, n, box)
    x0 = unwrapped(sysg.get_state(), s)
    deltas = []
    for k in range(1, 12):
        sysg.step(1)
        st = sysg.get_state()
        xw = wrapped(st, s, mc)
        acc, _ = oracle.forces(md, xw)
        events, worst = check_forces_at_cutoff(st["acc"], acc, xw, xw, box, 2.5)
        deltas.append(np.sqrt(((unwrapped(st, s) - x0) ** 2).sum(1)).max())
        say(f"  step {k}: largest displacement since the build {deltas[-1]:.4f} (skin {m:.4f}); "
            f"raw error {worst:.2e}, {events} at a cutoff pair")
        # (a pair within float rounding of r_c counts for both its particles)
        assert events <= 4
    assert max(deltas) > m / 2
    say(f"  force launches that walked the cells: {sysg.list_fallbacks()}")


# ------------------------------------------------------------------ autotuner

def test_autotuned_layout_runs_the_same_trajectory():
    import torch

    from paper_1705_04368_amd import autotune, describe
    cfg, pos, vel, box, n, M = _force_case(2, 79, 0, equil_steps=300)
    say("autotune")
    d = torch.device("cuda:0")
    best, ms = autotune(cfg, torch.from_numpy(pos).to(d), torch.from_numpy(vel).to(d), md_steps=40)
    lay = describe(best)
    say(f"  tuned {lay} at {ms * 1e3:.2f} us per MD step")
    assert ms > 0
    sysg = make_system(best, pos, vel)
    sysg.step(20)
    st = sysg.get_state()
    md = oracle.make_md(2, n, box, dt=0.005)
    ost = oracle.OracleState(md, pos, vel)
    ost.run(20)
    assert np.abs(unwrapped(st, lay["cell_side"]) - ost.unwrapped).max() <= 1e-4
    assert np.abs(st["vel"].astype(np.float64) - ost.v).max() <= 1e-4
