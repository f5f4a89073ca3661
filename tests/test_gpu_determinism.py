"""Determinism and checkpoints of the HIP path, with forces on.

The counting sort fixes every particle's slot from the previous order alone
(stayers first in their old order, then arrivals by direction and old order),
and the pair-list builder orders its targets stably, so no floating-point sum
depends on the order in which atomics land.  Hence, bit for bit:

* two runs from one state (2D and 3D with pair lists, 2D walking the cells,
  thermostatted steps, lattice steps, the collision operator and a moving
  lattice on);
* graph replay and eager launches;
* a batch of replicas and the same replicas run one by one;
* T lattice steps and T/2, checkpoint, load into another handle, T/2 (at a
  rebuild and between rebuilds, where the pair lists travel in the blob).
"""
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import make_system, say

pytestmark = pytest.mark.gpu

STATE_KEYS = ("ucell", "off", "vel", "acc", "prev_ucell", "prev_off")


def _cfg(dim=2, n=(2048,), lat=(16,), steps=20, pair_list=True, xi=False, shifts=None, **kw):
    from paper_1705_04368_amd import make_config
    return make_config(dim, list(n), [[m] * dim for m in lat], lattice_dx=4.0,
                       dt=0.005 if dim == 2 else 0.004, md_steps_per_lattice_step=steps,
                       vmax=3 if dim == 2 else 2, thermostat_every=10, kT=1.0 if dim == 2 else 1.5,
                       pair_list=pair_list, collision_stats=xi, shifts=shifts, **kw)


def _state(dim, n, lat, seed):
    ps, vs = [], []
    for r, (nr, m) in enumerate(zip(n, lat)):
        p, v = synth.lj_initial_state(dim, nr, 4.0 * m, 1.0 if dim == 2 else 1.5, seed=seed + r)
        ps.append(p)
        vs.append(v)
    return np.concatenate(ps), np.concatenate(vs)


def _run(cfg, pos, vel, thermo=30, T=3, graph=True):
    old = os.environ.get("MDLG_NO_GRAPH")
    os.environ["MDLG_NO_GRAPH"] = "0" if graph else "1"
    try:
        s = make_system(cfg, pos, vel)
    finally:
        if old is None:
            os.environ.pop("MDLG_NO_GRAPH", None)
        else:
            os.environ["MDLG_NO_GRAPH"] = old
    s.step(thermo)
    s.coarse_grain(T)
    return s


def _readout(s):
    out = {"f": s.get_f(per_site=True), "state": s.get_state(), "kin": s.kinetics()}
    if int(s.cfg.collision_stats):
        out["xi"] = s.get_xi(per_site=True, last=True)
    if int(s.cfg.n_shifts):
        out["shifts"] = s.get_shifts()
    return out


def _assert_same(a, b):
    for key in ("f_site", "mom_site", "counts", "disp_sum", "disp_sq"):
        np.testing.assert_array_equal(a["f"][key], b["f"][key], err_msg=key)
    assert a["f"]["n_lattice_steps"] == b["f"]["n_lattice_steps"]
    for key in STATE_KEYS:
        np.testing.assert_array_equal(a["state"][key], b["state"][key], err_msg=key)
    np.testing.assert_array_equal(a["kin"], b["kin"])
    if "xi" in a:
        for key in ("xi", "xi2", "xi_n", "n", "n2", "xi_site", "xi_last"):
            np.testing.assert_array_equal(a["xi"][key], b["xi"][key], err_msg=key)
        assert a["xi"]["n_steps"] == b["xi"]["n_steps"]
    if "shifts" in a:
        np.testing.assert_array_equal(a["shifts"]["counts"], b["shifts"]["counts"])
        np.testing.assert_array_equal(a["shifts"]["moments"], b["shifts"]["moments"])


@pytest.mark.parametrize("dim,pair_list", [(2, True), (2, False), (3, True)])
def test_identical_runs_bitwise(dim, pair_list):
    n, lat = ((2048,), (16,)) if dim == 2 else ((4740,), (5,))
    say(f"identical runs dim={dim} pair_list={pair_list}")
    sh = np.zeros((1, 2, dim))
    sh[0, 1, 0] = 0.25
    cfg = _cfg(dim, n, lat, pair_list=pair_list, xi=True, shifts=sh)
    pos, vel = _state(dim, n, lat, seed=401)
    a = _readout(_run(cfg, pos, vel))
    b = _readout(_run(cfg, pos, vel))
    _assert_same(a, b)
    # the run moved particles across cells (the slots are not trivially fixed)
    assert np.any(a["state"]["ucell"] != a["state"]["prev_ucell"]) or a["f"]["n_lattice_steps"] == 3


def test_graph_replay_equals_eager_with_forces():
    say("graph vs eager, forces on")
    sh = np.zeros((1, 2, 2))
    sh[0, 1, 0] = 0.25
    cfg = _cfg(xi=True, shifts=sh)
    pos, vel = _state(2, (2048,), (16,), seed=411)
    a = _readout(_run(cfg, pos, vel, graph=True, T=4))
    b = _readout(_run(cfg, pos, vel, graph=False, T=4))
    _assert_same(a, b)


def test_long_lattice_steps_graph_blocks_with_forces():
    # 450 MD steps per lattice step replay as graphs of whole rebuild
    # intervals plus a tail with the binning
    say("long lattice steps: block graphs vs eager, forces on")
    cfg = _cfg(steps=450, xi=True, sort_every=9)
    pos, vel = _state(2, (2048,), (16,), seed=417)
    a = _readout(_run(cfg, pos, vel, graph=True, T=2, thermo=20))
    b = _readout(_run(cfg, pos, vel, graph=False, T=2, thermo=20))
    _assert_same(a, b)


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_equals_separate_with_forces(dim):
    if dim == 2:
        sizes, lats = (968, 2048, 1568), (11, 16, 14)
        kw = dict(md_cell_split=1, sort_every=10, brick=(8, 2, 1), block_threads=128)
    else:
        # rho = 0.593 on lattices of 4, 5 and 6 cells of 4 sigma (partial bricks)
        sizes, lats = (2429, 4744, 8198), (4, 5, 6)
        kw = dict(md_cell_split=2, sort_every=10, brick=(4, 3, 3), block_threads=256)
    say(f"batched vs separate replicas, forces on, {dim}D")
    pos, vel = _state(dim, sizes, lats, seed=421)
    both = _run(_cfg(dim, sizes, lats, **kw), pos, vel)
    fb, sb, kb = both.get_f(per_site=True), both.get_state(), both.kinetics()
    p0, s0 = 0, 0
    for r, (n, m) in enumerate(zip(sizes, lats)):
        one = _run(_cfg(dim, (n,), (m,), **kw), pos[p0:p0 + n], vel[p0:p0 + n])
        f1, s1 = one.get_f(per_site=True), one.get_state()
        ns = m ** dim
        np.testing.assert_array_equal(fb["f_site"][s0:s0 + ns], f1["f_site"])
        np.testing.assert_array_equal(fb["mom_site"][s0:s0 + ns], f1["mom_site"])
        for key in STATE_KEYS:
            np.testing.assert_array_equal(sb[key][p0:p0 + n], s1[key], err_msg=key)
        np.testing.assert_array_equal(kb[r], one.kinetics()[0])
        p0 += n
        s0 += ns


@pytest.mark.parametrize("dim,extra_steps,batch", [(2, 0, False), (2, 7, False), (3, 0, False),
                                                   (2, 7, True)])
def test_checkpoint_resume_bitwise(dim, extra_steps, batch):
    # extra_steps: plain MD steps before the checkpoint, so that it is taken
    # between cell-list rebuilds (the pair lists travel in the blob); batch:
    # three replicas of different lattices in one handle
    if batch:
        n, lat = (968, 2048, 1568), (11, 16, 14)
    else:
        n, lat = ((2048,), (16,)) if dim == 2 else ((4740,), (5,))
    say(f"checkpoint dim={dim} extra_steps={extra_steps} replicas={len(n)}")
    sh = np.zeros((1, 2, dim))
    sh[0, 1, 0] = 0.25
    cfg = _cfg(dim, n, lat, xi=True, shifts=sh)
    pos, vel = _state(dim, n, lat, seed=431)
    full = _run(cfg, pos, vel, T=2)
    if extra_steps:
        full.step(extra_steps)
    full.coarse_grain(2)
    ref = _readout(full)
    half = _run(cfg, pos, vel, T=2)
    if extra_steps:
        half.step(extra_steps)
    blob = half.checkpoint()
    # another handle of the same configuration, started from another state
    pos2, vel2 = _state(dim, n, lat, seed=97)
    other = make_system(cfg, pos2, vel2)
    other.coarse_grain(1)
    other.restore(blob)
    other.coarse_grain(2)
    _assert_same(ref, _readout(other))
    # the blob is complete: loading it again into the first half's handle too
    half.restore(blob)
    half.coarse_grain(2)
    _assert_same(ref, _readout(half))


def test_checkpoint_rejects_other_configuration():
    from paper_1705_04368_amd import MdlgError
    say("checkpoint of another configuration")
    pos, vel = _state(2, (2048,), (16,), seed=441)
    a = make_system(_cfg(), pos, vel)
    blob = a.checkpoint()
    b = make_system(_cfg(steps=40), pos, vel)
    with pytest.raises(MdlgError, match="different configuration"):
        b.restore(blob)
    bad = blob.copy()
    bad[:8] = 0
    with pytest.raises(MdlgError, match="not an MDLG checkpoint"):
        a.restore(bad)
    with pytest.raises(MdlgError):
        a.restore(blob[:-8])


def test_sorted_layout_is_a_permutation_in_cell_order():
    # white-box check of the counting sort through the checkpoint blob, which
    # holds the state in the library's order: a header of 88 bytes, then
    # offsets, velocities, images, ids, cells, snapshot, cell starts
    for dim, n, lat in ((2, (968, 2048), (11, 16)), (3, (4740,), (5,))):
        say(f"sorted layout dim={dim}")
        cfg = _cfg(dim, n, lat)
        pos, vel = _state(dim, n, lat, seed=451)
        s = _run(cfg, pos, vel, thermo=40, T=3)
        blob = s.checkpoint()
        N = int(sum(n))
        off = 88
        take = {}
        for name, cnt, dt in (("pos", N * dim, np.float32), ("vel", N * dim, np.float32),
                              ("img", N * dim, np.int32), ("id", N, np.int32), ("cell", N, np.int32),
                              ("prev_u", N * dim, np.int32), ("prev_off", N * dim, np.float32),
                              ("cell_start", s.layout["n_cells"] + 1, np.int32)):
            nb = cnt * np.dtype(dt).itemsize
            take[name] = np.frombuffer(blob[off:off + nb].tobytes(), dtype=dt)
            off += nb
        np.testing.assert_array_equal(np.sort(take["id"]), np.arange(N))
        cell = take["cell"]
        assert np.all(np.diff(cell) >= 0)
        cs = take["cell_start"]
        np.testing.assert_array_equal(cs, np.searchsorted(cell, np.arange(len(cs)), side="left"))
        side = s.layout["cell_side"]
        p = take["pos"]
        assert np.all(p >= 0) and np.all(p < side)
        # every particle of a replica sits in a cell of that replica
        k = s.layout["md_cell_split"]
        bounds = np.concatenate([[0], np.cumsum(n)])
        cbounds = np.concatenate([[0], np.cumsum([(m * k) ** dim for m in lat])])
        for r in range(len(n)):
            c = cell[bounds[r]:bounds[r + 1]]
            assert c.min() >= cbounds[r] and c.max() < cbounds[r + 1]
            ids = take["id"][bounds[r]:bounds[r + 1]]
            assert ids.min() >= bounds[r] and ids.max() < bounds[r + 1]
