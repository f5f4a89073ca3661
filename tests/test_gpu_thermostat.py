"""The FP64 reductions and the equilibration thermostat against the oracle.

The paper sets the temperature of its LJ run by the kinetic energy and
discards the start of the run as equilibration (section "MDLG for a
two-dimensional Lennard-Jones gas"); the library equilibrates by rescaling
the velocities of every replica to sum m v^2 = kT d (N_r - 1) every
thermostat_every MD steps.  Bars:

* a thermostatted trajectory of 40 MD steps (four rescales) from one
  equilibrated state: |x_gpu - x_ref| <= 1e-4 sigma (unwrapped) and
  |v_gpu - v_ref| <= 1e-4 sqrt(kT/m) against the FP64 oracle's thermostatted
  velocity Verlet, for one system and for a batch of two replicas (each
  replica rescaled by its own factor, the oracle running each alone), in 2D
  and for a batch of two 3D replicas;
* mdlg_get_kinetics (FP64 momentum and kinetic energy per replica) against
  the oracle's sums over the GPU's own velocities: kinetic energy within
  1e-12 relative, momentum within 1e-12 of sum m |v|;
* right after a rescale, sum m v^2 / (d (N - 1)) = kT to float rounding.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import make_system, say, unwrapped

pytestmark = pytest.mark.gpu

KT, DT = 1.0, 0.005
# the 3D gas: kT = 1.5, dt = 0.004 at rho = 0.593
KT3, DT3 = 1.5, 0.004


def _equilibrated(n, M, seed, dim=2):
    """An oracle-equilibrated state (300 thermostatted steps) in [0, box)."""
    kT, dt = (KT, DT) if dim == 2 else (KT3, DT3)
    box = 4.0 * M
    pos, vel = synth.lj_initial_state(dim, n, box, kT, seed=seed)
    st = oracle.OracleState(oracle.make_md(dim, n, box, dt=dt), pos, vel)
    st.run(300, thermo_every=10, kT=kT)
    p = st.x.astype(np.float32)
    p = np.where(p >= np.float32(box), np.float32(0.0), p)
    return p, st.v.astype(np.float32)


def _cfg(sizes, lats, dim=2):
    from paper_1705_04368_amd import make_config
    kT, dt = (KT, DT) if dim == 2 else (KT3, DT3)
    return make_config(dim, list(sizes), [[m] * dim for m in lats], lattice_dx=4.0, dt=dt,
                       md_steps_per_lattice_step=20, vmax=3 if dim == 2 else 2,
                       thermostat_every=10, kT=kT)


@pytest.mark.parametrize("dim,sizes,lats", [(2, (2048,), (16,)), (2, (968, 1568), (11, 14)),
                                            (3, (2429, 4744), (4, 5))],
                         ids=["one", "two_replicas", "3d_two_replicas"])
def test_thermostatted_trajectory_matches_oracle(dim, sizes, lats):
    say(f"thermostatted trajectory {dim}D {sizes}")
    kT, dt = (KT, DT) if dim == 2 else (KT3, DT3)
    parts = [_equilibrated(n, m, seed=510 + r, dim=dim) for r, (n, m) in enumerate(zip(sizes, lats))]
    pos = np.concatenate([p for p, _ in parts])
    vel = np.concatenate([v for _, v in parts])
    sysg = make_system(_cfg(sizes, lats, dim), pos, vel)
    sysg.step(40)
    st = sysg.get_state()
    s = sysg.layout["cell_side"]
    xu = unwrapped(st, s)
    off = 0
    for (p, v), n, m in zip(parts, sizes, lats):
        box = 4.0 * m
        ost = oracle.OracleState(oracle.make_md(dim, n, box, dt=dt), p, v)
        ost.run(40, thermo_every=10, kT=kT)
        dx = np.abs(xu[off:off + n] - ost.unwrapped).max()
        dv = np.abs(st["vel"][off:off + n].astype(np.float64) - ost.v).max()
        say(f"  replica N={n}: max |dx| {dx:.2e}, max |dv| {dv:.2e}")
        assert dx <= 1e-4
        assert dv <= 1e-4 * np.sqrt(kT)
        # rescaled at the last step: the temperature is kT exactly
        t = np.sum(st["vel"][off:off + n].astype(np.float64) ** 2) / (dim * (n - 1))
        assert abs(t - kT) < 1e-5 * kT
        off += n


def test_kinetics_match_oracle_sums():
    sizes, lats = (968, 2048), (11, 16)
    say("kinetics against the oracle")
    parts = [_equilibrated(n, m, seed=530 + r) for r, (n, m) in enumerate(zip(sizes, lats))]
    pos = np.concatenate([p for p, _ in parts])
    vel = np.concatenate([v for _, v in parts])
    sysg = make_system(_cfg(sizes, lats), pos, vel)
    sysg.step(25)            # not at a rescale: the velocities are completed to full steps
    kin = sysg.kinetics()
    st = sysg.get_state()    # the same full-step velocities
    off = 0
    for r, (n, m) in enumerate(zip(sizes, lats)):
        v = st["vel"][off:off + n].astype(np.float64)
        ost = oracle.OracleState(oracle.make_md(2, n, 4.0 * m, dt=DT), parts[r][0], v)
        ke, mom = ost.kinetics()
        say(f"  replica {r}: KE gpu {kin[r, 2]:.15g} oracle {ke:.15g}; p gpu {kin[r, :2]} oracle {mom}")
        assert abs(kin[r, 2] - ke) <= 1e-12 * ke
        assert np.abs(kin[r, :2] - mom).max() <= 1e-12 * np.abs(v).sum()
        off += n
