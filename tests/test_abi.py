"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and validates configurations on the host (no device calls)."""
import ctypes as C
import os
import re

import pytest

from paper_1705_04368_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mdlg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdlg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = native.load()
    syms = declared_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(native.EXPORTED) == syms


def test_describe_config1():
    cfg = native.make_config(2, 2048, 16, lattice_dx=4.0, dt=0.005, md_steps_per_lattice_step=20,
                             vmax=3, kT=1.0)
    d = native.describe(cfg)
    assert d["n_velocities"] == 49
    assert d["n_moments"] == 7
    assert d["n_sites"] == 256
    assert d["n_total"] == 2048
    k = d["md_cell_split"]
    assert k in (1, 2, 4, 8)
    assert d["n_cells"] == 256 * k * k
    assert d["cell_side"] == 4.0 / k
    assert d["stencil"] * d["cell_side"] >= 2.5
    assert d["margin"] > 0
    assert 1 <= d["sort_every"] <= 20
    assert native.workspace_bytes(cfg) > 2048 * 2 * 4 * 4
    # the cell walk's reach: the excursion the one-cell halo still covers
    # when two particles, each that far outside its cell, are r_cut apart
    assert d["reach"] == pytest.approx((d["stencil"] * d["cell_side"] - 2.5) / 2, rel=1e-12)
    assert d["skin"] <= d["margin"] <= d["reach"] < d["cell_side"] / 2


def test_reach_is_independent_of_the_rebuild_interval():
    # the margin grows with the interval up to the reach; the reach does not
    lays = [native.describe(native.make_config(2, 2048, 16, lattice_dx=4.0, dt=0.005,
                                               md_cell_split=1, kT=1.0, sort_every=r))
            for r in (2, 10, 18, 40)]
    assert len({d["reach"] for d in lays}) == 1
    margins = [d["margin"] for d in lays]
    assert margins == sorted(margins) and margins[-1] == lays[0]["reach"]


def test_describe_3d_and_replicas():
    cfg = native.make_config(3, 4194304, 48, lattice_dx=4.0, dt=0.004, vmax=2, kT=1.5)
    d = native.describe(cfg)
    assert d["n_velocities"] == 125 and d["n_moments"] == 11 and d["n_sites"] == 48 ** 3
    cfg = native.make_config(2, [968, 2048, 66248], [[11, 11], [16, 16], [91, 91]], vmax=3)
    d = native.describe(cfg)
    assert d["n_total"] == 968 + 2048 + 66248
    assert d["n_sites"] == 121 + 256 + 8281


@pytest.mark.parametrize("change,msg", [
    (dict(dim=4), "dim"),
    (dict(vmax=8), "vmax"),
    (dict(dt=0.0), "dt"),
    (dict(md_cell_split=3), "power of two"),
    (dict(r_cut=40.0), "box side"),
    (dict(thermostat_every=5, kT=0.0), "kT"),
    (dict(md_steps_per_lattice_step=0), "md_steps"),
])
def test_invalid_configs_rejected(change, msg):
    kw = dict(dim=2, n_particles=100, lattice=8, lattice_dx=4.0)
    kw.update({k: v for k, v in change.items() if k in ("dim",)})
    extra = {k: v for k, v in change.items() if k != "dim"}
    cfg = native.make_config(kw["dim"], kw["n_particles"], 8, lattice_dx=4.0, **extra)
    with pytest.raises(native.MdlgError) as e:
        native.describe(cfg)
    assert e.value.status == -1
    assert msg in str(e.value)


def test_overfull_md_cells_rejected():
    # the hot dilute gas (N = 100000 in a 1000 sigma box, 10^2 lattice of
    # 100 sigma): one or two MD cells per lattice cell hold 1000 or 250
    # particles on average, beyond the counting sort's window; four hold 62.5
    def cfg(k):
        return native.make_config(2, 100000, 10, lattice_dx=100.0, dt=1e-4, kT=50.0, vmax=3,
                                  md_steps_per_lattice_step=341600, md_cell_split=k)
    for k in (1, 2):
        with pytest.raises(native.MdlgError, match="counting sort") as e:
            native.describe(cfg(k))
        assert e.value.status == -1
    for k in (0, 4, 8):
        assert native.describe(cfg(k))["md_cell_split"] in (4, 8)


def test_brick_halo_extent_bounded_by_the_map_packing():
    # a staging-map entry packs a halo cell in 8 bits per axis in 2D and 5 in
    # 3D: wider halos are refused (the halo-cell count alone allows them)
    def cfg2(bx):
        return native.make_config(2, 80000, 100, lattice_dx=4.0, md_cell_split=1, brick=(bx, 1, 1))
    assert native.describe(cfg2(254))["brick"] == (254, 1, 1)
    with pytest.raises(native.MdlgError, match="halo wider than 256") as e:
        native.describe(cfg2(255))
    assert e.value.status == -1

    def cfg3(bx):
        return native.make_config(3, 4740, 5, lattice_dx=4.0, vmax=1, md_cell_split=1,
                                  brick=(bx, 2, 2))
    assert native.describe(cfg3(30))["brick"] == (30, 2, 2)
    with pytest.raises(native.MdlgError, match="halo wider than 32"):
        native.describe(cfg3(31))


def test_vmax_window_limit_3d():
    cfg = native.make_config(3, 1000, 8, vmax=3)
    with pytest.raises(native.MdlgError, match="velocity window"):
        native.describe(cfg)


def test_create_rejects_null_inputs_without_device():
    lib = native.load()
    cfg = native.make_config(2, 100, 8)
    h = C.c_void_p(0)
    st = lib.mdlg_create(C.byref(cfg), None, 0, None, None, None, C.byref(h))
    assert st == -1
    assert b"required" in lib.mdlg_last_error(None)
    assert not h.value
    # misaligned workspace is rejected before any device call
    st = lib.mdlg_create(C.byref(cfg), C.c_void_p(0x1001), 1 << 20, None, C.c_void_p(0x2000),
                         C.c_void_p(0x3000), C.byref(h))
    assert st == -1 and b"aligned" in lib.mdlg_last_error(None)


def test_too_small_workspace_rejected():
    lib = native.load()
    cfg = native.make_config(2, 100, 8)
    h = C.c_void_p(0)
    st = lib.mdlg_create(C.byref(cfg), C.c_void_p(0x10000), 1024, None, C.c_void_p(0x2000),
                         C.c_void_p(0x3000), C.byref(h))
    assert st == -3
    assert b"too small" in lib.mdlg_last_error(None)


def test_null_handle_calls_are_invalid():
    lib = native.load()
    assert lib.mdlg_step(None, 1) == -1
    assert lib.mdlg_coarse_grain(None, 1) == -1
    assert lib.mdlg_sync(None) == -1
    v = C.c_double(0.0)
    assert lib.mdlg_timing_offset(None, 10, C.byref(v)) == -1
    assert lib.mdlg_timing_head_start(None, 10.0) == -1
    n = C.c_int64(0)
    assert lib.mdlg_get_list_fallbacks(None, C.byref(n)) == -1
    lib.mdlg_destroy(None)
