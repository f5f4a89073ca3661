"""Pins for the oracle's adjoint of a velocity-Verlet window (CPU only).

The reverse sweep is checked against central finite differences of the
forward loss (h = 1e-4 relative for eps and sigma, and along random directions
in v0-space), its pair terms against finite differences of the acceleration,
and the exact special cases: total momentum is conserved by velocity Verlet,
so the mean x displacement is W h <v0_x> independently of eps and sigma
(gradients 0 and W h / N); without forces the per-axis MSD is
(W h)^2 <|v0|^2> / d, whose gradient is 2 (W h)^2 v0 / (N d).
"""
import numpy as np
import pytest

import oracle
import synth

W, H = 20, 0.005


def _state(dim, n, box, seed, kT=1.0):
    pos, vel = synth.lj_initial_state(dim, n, box, kT, seed=seed)
    md = oracle.make_md(dim, n, box, dt=H)
    st = oracle.OracleState(md, pos, vel)
    st.run(200, thermo_every=10, kT=kT)  # leave the jittered grid
    return md, st.x.copy(), st.v.copy()


@pytest.mark.parametrize("dim,n,box", [(2, 64, 11.4), (3, 96, 5.5)])
def test_pair_terms_against_finite_differences(dim, n, box):
    md, x, _ = _state(dim, n, box, seed=3)
    rng = np.random.default_rng(0)
    lam = rng.normal(size=x.shape)
    acc, dacc, jl = oracle.pair_terms(md, x, lam)
    h = 1e-6
    ap, _, _ = oracle.pair_terms(md, x + h * lam)
    am, _, _ = oracle.pair_terms(md, x - h * lam)
    np.testing.assert_allclose(jl, (ap - am) / (2 * h), rtol=1e-5, atol=1e-5 * np.abs(jl).max())
    s0 = md.sigma
    md.sigma = s0 + 1e-6
    sp, _, _ = oracle.pair_terms(md, x)
    md.sigma = s0 - 1e-6
    sm, _, _ = oracle.pair_terms(md, x)
    md.sigma = s0
    np.testing.assert_allclose(dacc, (sp - sm) / 2e-6, rtol=1e-5, atol=1e-5 * np.abs(dacc).max())
    brute, _ = oracle.forces(md, x, brute=True)
    np.testing.assert_allclose(acc, brute, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("dim,n,box", [(2, 64, 11.4), (3, 96, 5.5)])
@pytest.mark.parametrize("loss", ["msd", "mean_x"])
def test_adjoint_matches_finite_differences(dim, n, box, loss):
    md, x0, v0 = _state(dim, n, box, seed=11 + dim)
    g = oracle.adjoint(md, x0, v0, W, loss)
    assert g["L"] == pytest.approx(oracle.window_loss(md, x0, v0, W, loss), rel=1e-14)
    # The forces are truncated at r_c, so the loss is only piecewise smooth:
    # a finite-difference interval in which a pair crosses the cutoff at some
    # step picks up the jump.  Gate at the 1e-3 bar with h = 1e-4 (relative),
    # and require convergence to 1e-6 at h = 1e-5.
    for name in ("eps", "sigma"):
        p0 = getattr(md, name)
        fds = []
        for rel in (1e-4, 1e-5):
            h = rel * p0
            setattr(md, name, p0 + h)
            lp = oracle.window_loss(md, x0, v0, W, loss)
            setattr(md, name, p0 - h)
            lm = oracle.window_loss(md, x0, v0, W, loss)
            setattr(md, name, p0)
            fds.append((lp - lm) / (2 * h))
        floor = 1e-8 * max(abs(g["L"]), 1e-3) / p0  # FP64 round-off of the loss over h
        assert abs(g[name] - fds[0]) <= 1e-3 * abs(fds[0]) + floor, (name, g[name], fds)
        assert abs(g[name] - fds[1]) <= 1e-6 * abs(fds[1]) + floor, (name, g[name], fds)
    rng = np.random.default_rng(1)
    for _ in range(4):
        u = rng.normal(size=v0.shape)
        u /= np.linalg.norm(u)
        h = 1e-4
        fd = (oracle.window_loss(md, x0, v0 + h * u, W, loss)
              - oracle.window_loss(md, x0, v0 - h * u, W, loss)) / (2 * h)
        ad = float(np.sum(g["v0"] * u))
        assert abs(ad - fd) <= 1e-3 * max(abs(fd), 1e-12) + 1e-12, (ad, fd)


def test_mean_displacement_gradients_are_exact():
    md, x0, v0 = _state(2, 256, 22.63, seed=5)
    g = oracle.adjoint(md, x0, v0, W, "mean_x")
    n = 256
    assert g["L"] == pytest.approx(W * H * v0[:, 0].mean(), abs=1e-12)
    assert abs(g["eps"]) < 1e-12 and abs(g["sigma"]) < 1e-12
    np.testing.assert_allclose(g["v0"][:, 0], W * H / n, rtol=1e-10)
    np.testing.assert_allclose(g["v0"][:, 1], 0.0, atol=1e-14)


def test_free_flight_msd_gradient_is_exact():
    dim, n, box = 3, 200, 8.0
    pos, vel = synth.lj_initial_state(dim, n, box, 1.0, seed=7)
    md = oracle.make_md(dim, n, box, dt=H, forces_off=True)
    x0, v0 = pos.astype(np.float64), vel.astype(np.float64)
    g = oracle.adjoint(md, x0, v0, W, "msd")
    np.testing.assert_allclose(g["v0"], 2 * (W * H) ** 2 * v0 / (n * dim), rtol=1e-10, atol=1e-16)
    assert g["eps"] == 0.0 and g["sigma"] == 0.0
    assert g["L"] == pytest.approx((W * H) ** 2 * np.sum(v0 ** 2) / (n * dim), rel=1e-10)
