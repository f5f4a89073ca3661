"""Adjoint of an MD window on the GPU (FP32) against the FP64 oracle adjoint.

Bar: loss and gradients within 1e-3 relative of the oracle's (the oracle's
adjoint is itself pinned to central finite differences with h = 1e-4 and to
exact cases in tests/test_oracle_adjoint.py); dL/dv0 per particle within 1e-3
of the largest component.  Exact cases on the GPU: the mean x displacement
does not depend on eps and sigma (momentum conservation) and its v0 gradient
is W h / N; without forces dL_msd/dv0 = 2 (W h)^2 v0 / (N d).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, make_system, say

pytestmark = pytest.mark.gpu
W, K, H = 20, 5, 0.005


def _setup(dim, n, M, dx, seed, equil=200, forces_off=False):
    from paper_1705_04368_amd import make_config
    box = M * dx
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=seed)
    if equil and not forces_off:
        st = oracle.OracleState(oracle.make_md(dim, n, box, dt=H), pos, vel)
        st.run(equil, thermo_every=10, kT=1.0)
        pos = st.x.astype(np.float32)
        pos = np.where(pos >= np.float32(box), np.float32(0.0), pos)
        vel = st.v.astype(np.float32)
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=H, vmax=2 if dim == 3 else 3, kT=1.0,
                      forces_off=forces_off, adjoint_window=W, adjoint_every=K)
    md = oracle.make_md(dim, n, box, dt=H, forces_off=forces_off)
    return cfg, md, pos, vel


def _compare(sysg, md, pos, vel, loss, v0=None):
    import torch
    v0_np = vel if v0 is None else v0
    L, ge, gs, gv = sysg.adjoint(W, K, loss,
                                 v0=None if v0 is None else torch.from_numpy(v0).to(device()))
    ref = oracle.adjoint(md, pos.astype(np.float64), v0_np.astype(np.float64), W, loss)
    gv = gv.cpu().numpy().astype(np.float64)
    say(f"  L {L:.8g} / {ref['L']:.8g}  eps {ge:.6g} / {ref['eps']:.6g}  "
        f"sigma {gs:.6g} / {ref['sigma']:.6g}  v0 max err "
        f"{np.abs(gv - ref['v0']).max() / np.abs(ref['v0']).max():.2e}")
    return L, ge, gs, gv, ref


@pytest.mark.parametrize("dim,n,M,dx", [(2, 2048, 16, 4.0), (3, 4740, 5, 4.0)])
def test_adjoint_msd_matches_oracle(dim, n, M, dx):
    cfg, md, pos, vel = _setup(dim, n, M, dx, seed=40 + dim)
    say(f"adjoint msd dim={dim} N={n}")
    sysg = make_system(cfg, pos, vel)
    L, ge, gs, gv, ref = _compare(sysg, md, pos, vel, "msd")
    assert L == pytest.approx(ref["L"], rel=1e-3)
    assert ge == pytest.approx(ref["eps"], rel=1e-3)
    assert gs == pytest.approx(ref["sigma"], rel=1e-3)
    assert np.abs(gv - ref["v0"]).max() <= 1e-3 * np.abs(ref["v0"]).max()


@pytest.mark.parametrize("dim,n,M,dx", [(2, 2048, 16, 4.0), (3, 4740, 5, 4.0)])
def test_adjoint_on_window_lists_equals_cell_walk(dim, n, M, dx):
    # the window's force and reverse steps walk pair lists built at its start
    # where pair lists are on, the frozen cells where they are off; both
    # against the oracle, and against each other (same FP32 terms, summed in
    # another order).  In 3D at rho = 0.6 a brick's halo of positions and
    # adjoint velocities exceeds the reverse step's LDS chunk, so there the
    # reverse step walks the cells either way (its force steps use the lists).
    cfg_l, md, pos, vel = _setup(dim, n, M, dx, seed=60 + dim)
    cfg_c, *_ = _setup(dim, n, M, dx, seed=60 + dim)
    cfg_c.no_pair_list = 1
    say(f"adjoint lists vs cell walk dim={dim} N={n}")
    out = []
    for cfg in (cfg_l, cfg_c):
        sysg = make_system(cfg, pos, vel)
        L, ge, gs, gv, ref = _compare(sysg, md, pos, vel, "msd")
        assert ge == pytest.approx(ref["eps"], rel=1e-3)
        assert gs == pytest.approx(ref["sigma"], rel=1e-3)
        assert np.abs(gv - ref["v0"]).max() <= 1e-3 * np.abs(ref["v0"]).max()
        out.append((L, ge, gs, gv))
    (L1, e1, s1, g1), (L2, e2, s2, g2) = out
    assert L1 == pytest.approx(L2, rel=1e-4)
    assert e1 == pytest.approx(e2, rel=1e-4)
    assert s1 == pytest.approx(s2, rel=1e-4)
    assert np.abs(g1 - g2).max() <= 1e-4 * np.abs(g2).max()


def test_adjoint_with_given_v0_and_state_after_window():
    cfg, md, pos, vel = _setup(2, 2048, 16, 4.0, seed=8)
    sysg = make_system(cfg, pos, vel)
    v0 = (1.5 * vel).astype(np.float32)
    say("adjoint with v0")
    L, ge, gs, gv, ref = _compare(sysg, md, pos, vel, "msd", v0=v0)
    assert ge == pytest.approx(ref["eps"], rel=1e-3)
    assert np.abs(gv - ref["v0"]).max() <= 1e-3 * np.abs(ref["v0"]).max()
    # the system now sits at the end of the window
    st = sysg.get_state()
    o = oracle.OracleState(md, pos, v0)
    o.run(W)
    s = sysg.layout["cell_side"]
    xg = st["ucell"].astype(np.float64) * s + st["off"]
    assert np.abs(xg - o.unwrapped).max() < 1e-4


def test_adjoint_mean_x_exact():
    cfg, md, pos, vel = _setup(2, 2048, 16, 4.0, seed=9)
    sysg = make_system(cfg, pos, vel)
    say("adjoint mean_x")
    L, ge, gs, gv, ref = _compare(sysg, md, pos, vel, "mean_x")
    n = pos.shape[0]
    # scale of a non-zero parameter gradient of this system, for the zero checks
    _, ge_msd, gs_msd, _ = make_system(cfg, pos, vel).adjoint(W, K, "msd")
    assert abs(ge) <= 1e-4 * abs(ge_msd) and abs(gs) <= 1e-4 * abs(gs_msd)
    np.testing.assert_allclose(gv[:, 0], W * H / n, rtol=1e-4)
    assert np.abs(gv[:, 1]).max() <= 1e-4 * W * H / n
    assert L == pytest.approx(W * H * vel[:, 0].astype(np.float64).mean(), abs=1e-7)


def test_adjoint_free_flight_exact():
    cfg, md, pos, vel = _setup(3, 1000, 4, 4.0, seed=10, forces_off=True)
    sysg = make_system(cfg, pos, vel)
    say("adjoint free flight")
    L, ge, gs, gv = sysg.adjoint(W, K, "msd")
    gv = gv.cpu().numpy()
    exact = 2 * (W * H) ** 2 * vel.astype(np.float64) / (1000 * 3)
    # float32 positions resolve the displacement to ~1e-7 sigma
    assert np.abs(gv - exact).max() <= 1e-4 * np.abs(exact).max()
    assert ge == 0.0 and gs == 0.0


def test_adjoint_full_size_window():
    # 2D LJ, N = 65536 at rho = 0.5 in a 362.04 sigma box (90 x 90 lattice)
    from paper_1705_04368_amd import make_config
    from paper_1705_04368_amd import describe
    dim, n, M = 2, 65536, 90
    dx = 362.04 / M
    cfg = make_config(dim, n, M, lattice_dx=dx, dt=H, vmax=3, kT=1.0, thermostat_every=10,
                      adjoint_window=W, adjoint_every=K)
    lay = describe(cfg)
    box = M * lay["md_cell_split"] * lay["cell_side"]  # float32 cell side times cells
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=5)
    sysg = make_system(cfg, pos, vel)
    say("adjoint full size: equilibrate on the oracle side, compare")
    st = oracle.OracleState(oracle.make_md(dim, n, box, dt=H), pos, vel)
    st.run(100, thermo_every=10, kT=1.0)
    p = st.x.astype(np.float32)
    p = np.where(p >= np.float32(box), np.float32(0.0), p)
    v = st.v.astype(np.float32)
    s = sysg.layout["cell_side"]
    k = sysg.layout["md_cell_split"]
    u = np.floor(p.astype(np.float64) / s).astype(np.int32)
    off = (p.astype(np.float64) - u * s).astype(np.float32)
    top = off >= np.float32(s)  # rounded up to the cell side: next cell, offset 0
    u = np.where(top, (u + 1) % (M * k), u).astype(np.int32)
    off = np.where(top, np.float32(0.0), off).astype(np.float32)
    sysg.set_state(u, off, v)
    md = oracle.make_md(dim, n, box, dt=H)
    xw = (u.astype(np.float64) * s + off.astype(np.float64))
    L, ge, gs, gv = sysg.adjoint(W, K, "msd")
    ref = oracle.adjoint(md, xw, v.astype(np.float64), W, "msd")
    gv = gv.cpu().numpy().astype(np.float64)
    say(f"  eps {ge:.6g} / {ref['eps']:.6g} sigma {gs:.6g} / {ref['sigma']:.6g}")
    assert ge == pytest.approx(ref["eps"], rel=1e-3)
    assert gs == pytest.approx(ref["sigma"], rel=1e-3)
    assert np.abs(gv - ref["v0"]).max() <= 1e-3 * np.abs(ref["v0"]).max()
    assert k >= 1


def test_autograd_function_matches_direct_call():
    import torch

    from paper_1705_04368_amd.autograd import window_loss
    cfg, md, pos, vel = _setup(2, 2048, 16, 4.0, seed=12)
    sysg = make_system(cfg, pos, vel)
    v0 = torch.from_numpy(vel).to(device()).requires_grad_(True)
    eps = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    say("autograd")
    L = window_loss(sysg, v0, eps, sig, W, K, "msd")
    (2.0 * L).backward()
    ref = oracle.adjoint(md, pos.astype(np.float64), vel.astype(np.float64), W, "msd")
    assert float(L) == pytest.approx(ref["L"], rel=1e-3)
    assert float(eps.grad) == pytest.approx(2 * ref["eps"], rel=1e-3)
    assert float(sig.grad) == pytest.approx(2 * ref["sigma"], rel=1e-3)
    g = v0.grad.cpu().numpy()
    assert np.abs(g - 2 * ref["v0"]).max() <= 1e-3 * np.abs(2 * ref["v0"]).max()
    # the window is evaluated again from the same state
    L2 = window_loss(sysg, v0.detach(), eps.detach(), sig.detach(), W, K, "msd")
    assert float(L2) == pytest.approx(float(L), rel=1e-6)


def test_adjoint_graph_replay_equals_eager():
    # mdlg_adjoint and mdlg_step replay captured graphs; three windows in a
    # row (each leaves the system W steps on, cells rebuilt), with plain MD
    # steps and synchronisations between them, against the same calls
    # launched one by one: every loss and gradient bit for bit, every replay
    import os
    cfg, md, pos, vel = _setup(2, 2048, 16, 4.0, seed=61)
    say("adjoint: graph replay vs eager, three windows")
    outs = {}
    for graph in (True, False):
        old = os.environ.get("MDLG_NO_GRAPH")
        os.environ["MDLG_NO_GRAPH"] = "0" if graph else "1"
        try:
            sysg = make_system(cfg, pos, vel)
        finally:
            if old is None:
                os.environ.pop("MDLG_NO_GRAPH", None)
            else:
                os.environ["MDLG_NO_GRAPH"] = old
        res = []
        for _ in range(3):
            L, ge, gs, gv = sysg.adjoint(W, K, "msd", want_v0=True)
            res.append((L, ge, gs, gv.cpu().numpy().copy()))
            sysg.step(7)
            sysg.sync()
        res.append(sysg.get_state())
        outs[graph] = res
    for i in range(3):
        a, b = outs[True][i], outs[False][i]
        assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]
        np.testing.assert_array_equal(a[3], b[3])
    for key in ("ucell", "off", "vel"):
        np.testing.assert_array_equal(outs[True][3][key], outs[False][3][key])


def test_adjoint_batched_replicas():
    """Two replicas in one batch: the loss runs over all N = N_1 + N_2
    particles, so the loss and its eps and sigma gradients are the particle-
    weighted means of the replicas' own, and dL/dv0 of a replica's particles
    is N_r / N times that replica's own (each replica against the oracle
    adjoint of that replica alone)."""
    from paper_1705_04368_amd import make_config
    sizes, lats, dx = (968, 2048), (11, 16), 4.0
    parts = []
    for r, (n, m) in enumerate(zip(sizes, lats)):
        box = m * dx
        pos, vel = synth.lj_initial_state(2, n, box, 1.0, seed=90 + r)
        st = oracle.OracleState(oracle.make_md(2, n, box, dt=H), pos, vel)
        st.run(200, thermo_every=10, kT=1.0)
        p = st.x.astype(np.float32)
        p = np.where(p >= np.float32(box), np.float32(0.0), p)
        parts.append((p, st.v.astype(np.float32), oracle.make_md(2, n, box, dt=H)))
    say("adjoint of a batch of two replicas")
    cfg = make_config(2, list(sizes), [[m, m] for m in lats], lattice_dx=dx, dt=H, vmax=3, kT=1.0,
                      adjoint_window=W, adjoint_every=K)
    N = sum(sizes)
    for loss in ("msd", "mean_x"):
        # (a window leaves its system at the window's end: a fresh one each)
        sysg = make_system(cfg, np.concatenate([p for p, _, _ in parts]),
                           np.concatenate([v for _, v, _ in parts]))
        L, ge, gs, gv = sysg.adjoint(W, K, loss)
        gv = gv.cpu().numpy().astype(np.float64)
        refs = [oracle.adjoint(md, p.astype(np.float64), v.astype(np.float64), W, loss)
                for p, v, md in parts]
        wts = [n / N for n in sizes]
        ref_L = sum(w * r["L"] for w, r in zip(wts, refs))
        ref_e = sum(w * r["eps"] for w, r in zip(wts, refs))
        ref_s = sum(w * r["sigma"] for w, r in zip(wts, refs))
        ref_v = np.concatenate([w * r["v0"] for w, r in zip(wts, refs)])
        say(f"  {loss}: L {L:.8g} / {ref_L:.8g}  eps {ge:.6g} / {ref_e:.6g}  "
            f"sigma {gs:.6g} / {ref_s:.6g}")
        assert np.abs(gv - ref_v).max() <= 1e-3 * np.abs(ref_v).max()
        if loss == "msd":
            assert L == pytest.approx(ref_L, rel=1e-3)
            assert ge == pytest.approx(ref_e, rel=1e-3)
            assert gs == pytest.approx(ref_s, rel=1e-3)
        else:
            # momentum conservation: the mean x displacement does not depend
            # on eps and sigma; the loss against the oracle's
            assert L == pytest.approx(ref_L, rel=1e-3, abs=1e-6)
            assert abs(ge) <= 1e-6 and abs(gs) <= 1e-6
