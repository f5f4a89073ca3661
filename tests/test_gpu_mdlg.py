"""MDLG statistics on the GPU against the FP64 oracle (2D LJ, N = 2048,
64 sigma box, 16 x 16 lattice of 4 sigma cells, Delta t = 20 MD steps, V = 3).

* f_i: GPU FP32 and oracle FP64 runs from the same equilibrated state are
  independent estimates of <n_i> (eq. fieq); batch-means standard errors over
  blocks of lattice steps; the gate is a Sidak-adjusted family-wise 1% test
  over bins with at least 100 expected counts, plus at least 90% of those
  bins within 3 standard errors;
* the mass identity sum_i n_i + overflow = N(x,t) per site and in total, and
  the telescoping of the lattice momentum, exactly (integers).
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth
from paper_1705_04368_amd.native import MdlgError
from tests.gpu_util import make_system, say

pytestmark = pytest.mark.gpu

DIM, N, M, DX, KT, DT, V = 2, 2048, 16, 4.0, 1.0, 0.005, 3


@pytest.fixture(scope="module")
def equilibrated():
    box = M * DX
    pos, vel = synth.lj_initial_state(DIM, N, box, KT, seed=1)
    md = oracle.make_md(DIM, N, box, dt=DT)
    st = oracle.OracleState(md, pos, vel)
    say("oracle equilibration: 2000 steps")
    st.run(2000, thermo_every=10, kT=KT)
    p = st.x.astype(np.float32)
    p = np.where(p >= np.float32(box), np.float32(0.0), p)
    return p, st.v.astype(np.float32)


def _cfg(steps=20):
    from paper_1705_04368_amd import make_config
    return make_config(DIM, N, M, lattice_dx=DX, dt=DT, md_steps_per_lattice_step=steps, vmax=V,
                       kT=KT)


# Delta t = 20 MD steps (the configuration's), and 160 steps where collisions
# matter and the second shell of velocities fills
@pytest.mark.parametrize("STEPS,BLOCKS,PER_BLOCK", [(20, 20, 10), (160, 12, 5)])
def test_lj_fi_within_standard_errors(equilibrated, STEPS, BLOCKS, PER_BLOCK):
    pos, vel = equilibrated
    T = BLOCKS * PER_BLOCK
    say(f"oracle production: {T} lattice steps of {STEPS}")
    box = M * DX
    ost = oracle.OracleState(oracle.make_md(DIM, N, box, dt=DT), pos, vel)
    o = ost.mdlg(oracle.make_lattice(DIM, (M, M), DX, V), STEPS, T, per_step_hist=True)
    ob = o["hist"].astype(np.float64).reshape(BLOCKS, PER_BLOCK, -1).sum(axis=1) / (PER_BLOCK * M * M)
    say("gpu production")
    sysg = make_system(_cfg(STEPS), pos, vel)
    prev = np.zeros(sysg.Q)
    gb = []
    for b in range(BLOCKS):
        sysg.coarse_grain(PER_BLOCK)
        c = sysg.get_f()["counts"].astype(np.float64)
        gb.append((c - prev) / (PER_BLOCK * M * M))
        prev = c
    gb = np.array(gb)
    fg, fo = gb.mean(0), ob.mean(0)
    seg = gb.std(0, ddof=1) / math.sqrt(BLOCKS)
    seo = ob.std(0, ddof=1) / math.sqrt(BLOCKS)
    tested = fo * T * M * M >= 100
    z = (fg - fo)[tested] / np.sqrt(seg[tested] ** 2 + seo[tested] ** 2)
    m = int(tested.sum())
    thr = norm.isf((1 - (1 - 0.01) ** (1.0 / m)) / 2)
    say(f"  bins tested {m}, max |z| {np.abs(z).max():.2f} (Sidak threshold {thr:.2f}), "
        f"within 3 SE: {(np.abs(z) <= 3).sum()}/{m}")
    assert m >= 5
    assert np.abs(z).max() < thr
    assert (np.abs(z) <= 3).mean() >= 0.9
    # the same mass in both: sum_i f_i + overflow rate = N / sites exactly
    g = sysg.get_f()
    assert g["counts"].sum() + g["n_overflow"] == N * T


def test_mass_and_momentum_identities_on_lj_run(equilibrated):
    pos, vel = equilibrated
    sysg = make_system(_cfg(), pos, vel)
    k = sysg.layout["md_cell_split"]
    st0 = sysg.get_state()
    T = 30
    say("identities: 30 lattice steps")
    sysg.coarse_grain(T)
    g = sysg.get_f(per_site=True)
    st1 = sysg.get_state()
    A = np.rint(g["f_site"] * T).astype(np.int64)
    mom = np.rint(g["mom_site"] * T).astype(np.int64)
    rho, ovf = mom[:, 0], mom[:, 1]
    np.testing.assert_array_equal(A.sum(axis=1) + ovf, rho)
    assert rho.sum() == N * T
    net = (np.floor_divide(st1["ucell"], k) - np.floor_divide(st0["ucell"], k)).astype(np.int64).sum(0)
    np.testing.assert_array_equal(mom[:, 2:2 + DIM].sum(axis=0), net)
    # continuous displacement: telescopes to the net unwrapped displacement
    s = sysg.layout["cell_side"]
    x0 = st0["ucell"].astype(np.float64) * s + st0["off"]
    x1 = st1["ucell"].astype(np.float64) * s + st1["off"]
    np.testing.assert_allclose(g["disp_sum"], (x1 - x0).sum(0), rtol=1e-9, atol=1e-6)
    # FP64 momentum of the MD stays at its initial (zero) value
    kin = sysg.kinetics()
    assert np.abs(kin[0, :DIM]).max() < 1e-2
    assert abs(2 * kin[0, DIM] / (DIM * (N - 1)) - KT) < 0.2


def test_event_timing_offset(equilibrated):
    """mdlg_timing_offset: the constant an event pair adds, from a kernel that
    waits a known span of the device's wall clock.  Non-negative (the wait is
    never shorter than its span), a few microseconds, repeatable; per-launch
    timing of a lattice step is not disturbed by it."""
    pos, vel = equilibrated
    sysg = make_system(_cfg(), pos, vel)
    sysg.set_timing(True)
    # the launches of the pass are enqueued while the device waits 2 ms
    sysg.timing_head_start(2000)
    sysg.coarse_grain(2)
    tim = sysg.get_timing()
    for bad in (-1.0, 2e6):
        with pytest.raises(MdlgError):
            sysg.timing_head_start(bad)
    say("event offset: two measurements")
    o1 = sysg.timing_offset(50)
    o2 = sysg.timing_offset(50)
    assert sysg.get_timing() == tim
    sysg.set_timing(False)
    assert 0.0 <= o1 < 0.05 and 0.0 <= o2 < 0.05
    assert abs(o1 - o2) < 0.01
    assert tim["force"][1] == 40 and tim["force"][0] / 40 > o1
