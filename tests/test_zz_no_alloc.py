"""mdlg_create_static (the library's static device workspace, no allocation)
against mdlg_create (a caller workspace), through the C ABI.

The library is deterministic, so the two handles must agree bit for bit on
the particle state, the accumulators and the kinetics after thermostatted
steps and lattice steps.  Two calls in a row, the second with a smaller
system (the array keeps the first call's contents, which creation must clear
where it matters).  Also: a second static handle while one is alive is
refused (MDLG_E_STATE), and a configuration beyond the array's size is
refused (MDLG_E_NOMEM) before any device work.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import device, make_system, say

pytestmark = pytest.mark.gpu


def _cfg(n, M):
    from paper_1705_04368_amd import make_config
    return make_config(2, n, M, lattice_dx=4.0, dt=0.005, md_steps_per_lattice_step=20, vmax=3,
                       thermostat_every=10, kT=1.0, collision_stats=True)


def _readout(s):
    f = s.get_f(per_site=True)
    return f, s.get_state(), s.kinetics(), s.get_xi(per_site=True)


def _static_system(cfg, pos, vel):
    import torch

    from paper_1705_04368_amd import System
    d = device()
    return System(cfg, torch.from_numpy(pos).to(d), torch.from_numpy(vel).to(d), static=True)


def test_static_workspace_matches_caller_workspace():
    from paper_1705_04368_amd import MdlgError
    for n, M, seed in ((2048, 16, 701), (968, 11, 702)):
        say(f"static workspace N={n}")
        cfg = _cfg(n, M)
        pos, vel = synth.lj_initial_state(2, n, 4.0 * M, 1.0, seed=seed)
        st = _static_system(cfg, pos, vel)
        assert st.workspace is None
        with pytest.raises(MdlgError) as e:
            _static_system(cfg, pos, vel)
        assert e.value.status == -5
        ref = make_system(cfg, pos, vel)
        for s in (st, ref):
            s.step(30)
            s.coarse_grain(3)
        a, b = _readout(st), _readout(ref)
        for key in ("f_site", "mom_site", "counts", "disp_sum", "disp_sq"):
            np.testing.assert_array_equal(a[0][key], b[0][key], err_msg=key)
        for key in ("ucell", "off", "vel", "acc", "prev_ucell", "prev_off"):
            np.testing.assert_array_equal(a[1][key], b[1][key], err_msg=key)
        np.testing.assert_array_equal(a[2], b[2])
        for key in ("xi", "xi2", "xi_site"):
            np.testing.assert_array_equal(a[3][key], b[3][key], err_msg=key)
        st.close()
        ref.close()


def test_static_workspace_rejects_large_configuration():
    from paper_1705_04368_amd import MdlgError
    say("static workspace: configuration too large")
    n, M = 262144, 181
    pos = np.zeros((n, 2), np.float32)
    with pytest.raises(MdlgError) as e:
        _static_system(_cfg(n, M), pos, pos)
    assert e.value.status == -3 and "static workspace holds" in str(e.value)
