"""ctypes binding of libmdlg.so (include/mdlg.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory (the
workspace and the initial arrays) and the stream.  Loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdlg.so")

MDLG_OK = 0
STATUS = {0: "MDLG_OK", -1: "MDLG_E_INVALID", -2: "MDLG_E_DEVICE", -3: "MDLG_E_NOMEM",
          -4: "MDLG_E_UNSTABLE", -5: "MDLG_E_STATE"}

EXPORTED = ["mdlg_describe", "mdlg_workspace_bytes", "mdlg_create", "mdlg_step",
            "mdlg_coarse_grain", "mdlg_get_f", "mdlg_get_kinetics", "mdlg_reset_accumulators",
            "mdlg_get_state", "mdlg_set_state", "mdlg_adjoint", "mdlg_set_potential",
            "mdlg_set_timing", "mdlg_get_timing", "mdlg_sync", "mdlg_last_error", "mdlg_destroy",
            "mdlg_autotune", "mdlg_autotune_workspace_bytes", "mdlg_get_xi", "mdlg_get_shifts",
            "mdlg_checkpoint_bytes", "mdlg_checkpoint_save", "mdlg_checkpoint_load",
            "mdlg_create_static", "mdlg_get_list_fallbacks", "mdlg_timing_offset",
            "mdlg_timing_head_start"]
LOSSES = {"msd": 0, "mean_x": 1}
KERNEL_CLASSES = ["force", "count", "scan", "scatter", "bin", "nlist", "xi", "shift", "adjoint",
                  "adjoint_force"]


class MdlgConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_replicas", C.c_int32),
                ("n_particles", C.POINTER(C.c_int32)), ("lattice", C.POINTER(C.c_int32)),
                ("lattice_dx", C.c_double), ("epsilon", C.c_double), ("sigma", C.c_double),
                ("mass", C.c_double), ("r_cut", C.c_double), ("forces_off", C.c_int32),
                ("dt", C.c_double), ("md_steps_per_lattice_step", C.c_int32),
                ("vmax", C.c_int32), ("thermostat_every", C.c_int32), ("kT", C.c_double),
                ("md_cell_split", C.c_int32), ("sort_every", C.c_int32),
                ("brick_x", C.c_int32), ("brick_y", C.c_int32), ("brick_z", C.c_int32),
                ("adjoint_window", C.c_int32), ("adjoint_every", C.c_int32),
                ("no_pair_list", C.c_int32), ("block_threads", C.c_int32),
                ("collision_stats", C.c_int32), ("n_shifts", C.c_int32),
                ("shifts", C.POINTER(C.c_double))]


class MdlgParticles(C.Structure):
    _fields_ = [("ucell", C.POINTER(C.c_int32)), ("off", C.POINTER(C.c_float)),
                ("vel", C.POINTER(C.c_float)), ("acc", C.POINTER(C.c_float)),
                ("prev_ucell", C.POINTER(C.c_int32)), ("prev_off", C.POINTER(C.c_float))]


class MdlgLayout(C.Structure):
    _fields_ = [("md_cell_split", C.c_int32), ("sort_every", C.c_int32),
                ("stencil", C.c_int32), ("n_velocities", C.c_int32), ("n_moments", C.c_int32),
                ("brick", C.c_int32 * 3), ("n_total", C.c_int64), ("n_sites", C.c_int64),
                ("n_cells", C.c_int64), ("n_bricks", C.c_int64), ("cell_side", C.c_double),
                ("margin", C.c_double), ("pair_slots", C.c_int32), ("block_threads", C.c_int32),
                ("skin", C.c_double), ("reach", C.c_double)]


_lib = None


def library_path():
    return LIB_PATH


def load():
    """Load libmdlg.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1705_04368_amd.build")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    st = C.c_int
    lib.mdlg_describe.restype = st
    lib.mdlg_describe.argtypes = [P(MdlgConfig), P(MdlgLayout)]
    lib.mdlg_workspace_bytes.restype = st
    lib.mdlg_workspace_bytes.argtypes = [P(MdlgConfig), P(C.c_size_t)]
    lib.mdlg_create.restype = st
    lib.mdlg_create.argtypes = [P(MdlgConfig), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                C.c_void_p, P(C.c_void_p)]
    lib.mdlg_create_static.restype = st
    lib.mdlg_create_static.argtypes = [P(MdlgConfig), C.c_void_p, C.c_void_p, C.c_void_p,
                                       P(C.c_void_p)]
    lib.mdlg_step.restype = st
    lib.mdlg_step.argtypes = [C.c_void_p, C.c_int64]
    lib.mdlg_coarse_grain.restype = st
    lib.mdlg_coarse_grain.argtypes = [C.c_void_p, C.c_int64]
    lib.mdlg_get_f.restype = st
    lib.mdlg_get_f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               P(C.c_int64), P(C.c_int64), C.c_void_p, P(C.c_int64)]
    lib.mdlg_get_kinetics.restype = st
    lib.mdlg_get_kinetics.argtypes = [C.c_void_p, C.c_void_p]
    lib.mdlg_reset_accumulators.restype = st
    lib.mdlg_reset_accumulators.argtypes = [C.c_void_p]
    lib.mdlg_get_state.restype = st
    lib.mdlg_get_state.argtypes = [C.c_void_p, P(MdlgParticles)]
    lib.mdlg_set_state.restype = st
    lib.mdlg_set_state.argtypes = [C.c_void_p, P(MdlgParticles)]
    lib.mdlg_adjoint.restype = st
    lib.mdlg_adjoint.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 P(C.c_double), P(C.c_double), P(C.c_double), C.c_void_p]
    lib.mdlg_set_potential.restype = st
    lib.mdlg_set_potential.argtypes = [C.c_void_p, C.c_double, C.c_double]
    lib.mdlg_set_timing.restype = st
    lib.mdlg_set_timing.argtypes = [C.c_void_p, C.c_int]
    lib.mdlg_get_timing.restype = st
    lib.mdlg_get_timing.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.mdlg_timing_offset.restype = st
    lib.mdlg_timing_offset.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    lib.mdlg_timing_head_start.restype = st
    lib.mdlg_timing_head_start.argtypes = [C.c_void_p, C.c_double]
    lib.mdlg_get_list_fallbacks.restype = st
    lib.mdlg_get_list_fallbacks.argtypes = [C.c_void_p, C.c_void_p]
    lib.mdlg_sync.restype = st
    lib.mdlg_sync.argtypes = [C.c_void_p]
    lib.mdlg_last_error.restype = C.c_char_p
    lib.mdlg_last_error.argtypes = [C.c_void_p]
    lib.mdlg_destroy.restype = None
    lib.mdlg_destroy.argtypes = [C.c_void_p]
    lib.mdlg_autotune.restype = st
    lib.mdlg_autotune.argtypes = [P(MdlgConfig), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int32, P(MdlgConfig), P(C.c_double)]
    lib.mdlg_get_shifts.restype = st
    lib.mdlg_get_shifts.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_int64)]
    lib.mdlg_get_xi.restype = st
    lib.mdlg_get_xi.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_int64)]
    lib.mdlg_checkpoint_bytes.restype = st
    lib.mdlg_checkpoint_bytes.argtypes = [C.c_void_p, P(C.c_size_t)]
    lib.mdlg_checkpoint_save.restype = st
    lib.mdlg_checkpoint_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.mdlg_checkpoint_load.restype = st
    lib.mdlg_checkpoint_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.mdlg_autotune_workspace_bytes.restype = st
    lib.mdlg_autotune_workspace_bytes.argtypes = [P(MdlgConfig), P(C.c_size_t)]
    _lib = lib
    return lib


class MdlgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _check(status, handle=None):
    if status != MDLG_OK:
        msg = load().mdlg_last_error(handle)
        raise MdlgError(status, msg.decode() if msg else "")


def make_config(dim, n_particles, lattice, lattice_dx=4.0, epsilon=1.0, sigma=1.0, mass=1.0,
                r_cut=2.5, forces_off=False, dt=0.005, md_steps_per_lattice_step=20, vmax=3,
                thermostat_every=0, kT=1.0, md_cell_split=0, sort_every=0, brick=(0, 0, 0),
                adjoint_window=0, adjoint_every=1, pair_list=True, block_threads=0,
                collision_stats=False, shifts=None):
    """Build an MdlgConfig.  n_particles: int or sequence per replica; lattice:
    sites per axis, an int, a (dim,) sequence or an (n_replicas, dim) array."""
    n = np.atleast_1d(np.asarray(n_particles, dtype=np.int32))
    lat = np.asarray(lattice, dtype=np.int32)
    if lat.ndim == 0:
        lat = np.full((len(n), dim), int(lat), dtype=np.int32)
    elif lat.ndim == 1:
        lat = np.broadcast_to(lat, (len(n), dim)).astype(np.int32)
    n = np.ascontiguousarray(n)
    lat = np.ascontiguousarray(lat, dtype=np.int32)
    cfg = MdlgConfig()
    cfg.dim = dim
    cfg.n_replicas = len(n)
    cfg.n_particles = n.ctypes.data_as(C.POINTER(C.c_int32))
    cfg.lattice = lat.ctypes.data_as(C.POINTER(C.c_int32))
    cfg._keep = (n, lat)  # the arrays must outlive the struct
    cfg.lattice_dx = lattice_dx
    cfg.epsilon, cfg.sigma, cfg.mass, cfg.r_cut = epsilon, sigma, mass, r_cut
    cfg.forces_off = int(bool(forces_off))
    cfg.dt = dt
    cfg.md_steps_per_lattice_step = md_steps_per_lattice_step
    cfg.vmax = vmax
    cfg.thermostat_every = thermostat_every
    cfg.kT = kT
    cfg.md_cell_split = md_cell_split
    cfg.sort_every = sort_every
    cfg.brick_x, cfg.brick_y, cfg.brick_z = (int(b) for b in brick)
    cfg.adjoint_window = adjoint_window
    cfg.adjoint_every = adjoint_every if adjoint_window else 0
    cfg.no_pair_list = 0 if pair_list else 1
    cfg.block_threads = block_threads
    cfg.collision_stats = int(bool(collision_stats))
    keep = [n, lat]
    if shifts is not None:
        # [n_shifts][2][dim]: offset a and drift b per axis, in lattice spacings
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(-1, 2, dim))
        cfg.n_shifts = sh.shape[0]
        cfg.shifts = sh.ctypes.data_as(C.POINTER(C.c_double))
        keep.append(sh)
    cfg._keep = tuple(keep)
    return cfg


def describe(cfg):
    out = MdlgLayout()
    _check(load().mdlg_describe(C.byref(cfg), C.byref(out)))
    return {"md_cell_split": out.md_cell_split, "sort_every": out.sort_every,
            "stencil": out.stencil, "n_velocities": out.n_velocities,
            "n_moments": out.n_moments, "brick": tuple(out.brick), "n_total": out.n_total,
            "n_sites": out.n_sites, "n_cells": out.n_cells, "n_bricks": out.n_bricks,
            "cell_side": out.cell_side, "margin": out.margin, "pair_slots": out.pair_slots,
            "block_threads": out.block_threads, "skin": out.skin, "reach": out.reach}


def workspace_bytes(cfg):
    b = C.c_size_t(0)
    _check(load().mdlg_workspace_bytes(C.byref(cfg), C.byref(b)))
    return int(b.value)


def autotune(cfg, pos, vel, md_steps=100, stream=None):
    """Time candidate launch shapes of cfg on the device (mdlg_autotune) from
    the state pos, vel (float32 device tensors, as for System) and return
    (tuned config, ms per MD step).  Fields of cfg left at 0 are tuned."""
    import torch
    lib = load()
    b = C.c_size_t(0)
    _check(lib.mdlg_autotune_workspace_bytes(C.byref(cfg), C.byref(b)))
    nbytes = int(b.value)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=pos.device)
    aligned = (ws.data_ptr() + 255) & ~255
    if stream is None:
        stream = torch.cuda.current_stream(pos.device)
    pos = pos.contiguous()
    vel = vel.contiguous()
    best = MdlgConfig()
    ms = C.c_double(0.0)
    _check(lib.mdlg_autotune(C.byref(cfg), C.c_void_p(aligned), C.c_size_t(nbytes),
                             C.c_void_p(stream.cuda_stream), C.c_void_p(pos.data_ptr()),
                             C.c_void_p(vel.data_ptr()), int(md_steps), C.byref(best), C.byref(ms)))
    best._keep = getattr(cfg, "_keep", None)  # the replica arrays stay alive with the copy
    del ws
    return best, float(ms.value)


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class System:
    """One MDLG system (one or many replicas) on the current HIP device.

    pos, vel: torch float32 device tensors of shape (n_total, dim) holding the
    initial positions in [0, box) and velocities.  static: take the library's
    static device workspace (mdlg_create_static) instead of allocating one."""

    def __init__(self, cfg, pos, vel, stream=None, static=False):
        import torch
        lib = load()
        self.cfg = cfg
        self.layout = describe(cfg)
        self.dim = cfg.dim
        self.n_total = int(self.layout["n_total"])
        self.n_sites = int(self.layout["n_sites"])
        self.Q = int(self.layout["n_velocities"])
        self.nm = int(self.layout["n_moments"])
        if pos.dtype != torch.float32 or vel.dtype != torch.float32:
            raise TypeError("positions and velocities must be float32")
        if tuple(pos.shape) != (self.n_total, self.dim) or tuple(vel.shape) != (self.n_total, self.dim):
            raise ValueError(f"expected ({self.n_total}, {self.dim}) arrays")
        if not pos.is_cuda or not vel.is_cuda:
            raise ValueError("positions and velocities must be device tensors")
        self.device = pos.device
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._pos = pos.contiguous()
        self._vel = vel.contiguous()
        h = C.c_void_p(0)
        if static:
            self.workspace = None
            st = lib.mdlg_create_static(C.byref(cfg), C.c_void_p(stream.cuda_stream),
                                        C.c_void_p(self._pos.data_ptr()),
                                        C.c_void_p(self._vel.data_ptr()), C.byref(h))
        else:
            nbytes = workspace_bytes(cfg)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) & ~255
            st = lib.mdlg_create(C.byref(cfg), C.c_void_p(aligned), C.c_size_t(nbytes),
                                 C.c_void_p(stream.cuda_stream), C.c_void_p(self._pos.data_ptr()),
                                 C.c_void_p(self._vel.data_ptr()), C.byref(h))
        _check(st, None)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().mdlg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_shifts(self):
        """Histograms of the displaced / moving lattices (mdlg_get_shifts):
        counts [n_shifts, Q + 1] (window bins, then overflow), moments
        [n_shifts, d + d(d+1)/2] (sum of v_a, then v_a v_b) and n_steps."""
        ns = int(self.cfg.n_shifts)
        counts = np.zeros((ns, self.Q + 1), dtype=np.uint64)
        mom = np.zeros((ns, self.dim + self.dim * (self.dim + 1) // 2), dtype=np.int64)
        n = C.c_int64(0)
        _check(load().mdlg_get_shifts(self.handle, counts.ctypes.data_as(C.c_void_p),
                                      mom.ctypes.data_as(C.c_void_p), C.byref(n)), self.handle)
        return {"counts": counts, "moments": mom, "n_steps": int(n.value)}

    def get_xi(self, per_site=False, last=False):
        """Collision-operator statistics (mdlg_get_xi): dict with the number of
        samples, per-bin sums of Xi, Xi^2, Xi n, n, n^2 (int64 [Q] each), and
        optionally the per-site sums and the latest field ([n_sites, Q])."""
        sums = np.zeros((5, self.Q), dtype=np.int64)
        site = np.zeros((self.n_sites, self.Q), dtype=np.int64) if per_site else None
        lastf = np.zeros((self.n_sites, self.Q), dtype=np.int32) if last else None
        n = C.c_int64(0)
        _check(load().mdlg_get_xi(self.handle, sums.ctypes.data_as(C.c_void_p),
                                  None if site is None else site.ctypes.data_as(C.c_void_p),
                                  None if lastf is None else lastf.ctypes.data_as(C.c_void_p),
                                  C.byref(n)), self.handle)
        out = {"n_steps": int(n.value), "xi": sums[0], "xi2": sums[1], "xi_n": sums[2],
               "n": sums[3], "n2": sums[4]}
        if per_site:
            out["xi_site"] = site
        if last:
            out["xi_last"] = lastf
        return out

    def step(self, n):
        _check(load().mdlg_step(self.handle, int(n)), self.handle)

    def coarse_grain(self, n_lattice_steps):
        _check(load().mdlg_coarse_grain(self.handle, int(n_lattice_steps)), self.handle)

    def sync(self):
        _check(load().mdlg_sync(self.handle), self.handle)

    def adjoint(self, window, ckpt_every, loss="msd", v0=None, want_v0=True):
        """Loss of the displacement over `window` MD steps from the current
        positions (and v0, a device tensor in id order, when given) with its
        gradients: returns (L, dL/deps, dL/dsigma, dL/dv0 device tensor or None)."""
        import torch
        L, ge, gs = C.c_double(0), C.c_double(0), C.c_double(0)
        g = torch.empty((self.n_total, self.dim), dtype=torch.float32, device=self.device) if want_v0 else None
        if v0 is not None:
            v0 = v0.detach().to(device=self.device, dtype=torch.float32).contiguous()
        _check(load().mdlg_adjoint(self.handle, int(window), int(ckpt_every), LOSSES[loss],
                                   C.c_void_p(v0.data_ptr()) if v0 is not None else None,
                                   C.byref(L), C.byref(ge), C.byref(gs),
                                   C.c_void_p(g.data_ptr()) if g is not None else None), self.handle)
        return L.value, ge.value, gs.value, g

    def set_potential(self, epsilon, sigma):
        _check(load().mdlg_set_potential(self.handle, float(epsilon), float(sigma)), self.handle)

    def set_timing(self, enable):
        _check(load().mdlg_set_timing(self.handle, int(bool(enable))), self.handle)

    def get_timing(self):
        """{kernel class: (total ms, launches)} since timing was enabled."""
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        _check(load().mdlg_get_timing(self.handle, ms.ctypes.data_as(C.c_void_p),
                                      n.ctypes.data_as(C.c_void_p)), self.handle)
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def timing_offset(self, reps=50):
        """Milliseconds an event pair adds to a kernel's time (mdlg_timing_offset)."""
        v = C.c_double(0.0)
        _check(load().mdlg_timing_offset(self.handle, int(reps), C.byref(v)), self.handle)
        return float(v.value)

    def timing_head_start(self, microseconds):
        """Enqueue a device-side wait so that the launches after it run back to
        back (mdlg_timing_head_start)."""
        _check(load().mdlg_timing_head_start(self.handle, float(microseconds)), self.handle)

    def list_fallbacks(self):
        """Force launches that walked the cells for possibly stale pair lists."""
        n = C.c_int64(0)
        _check(load().mdlg_get_list_fallbacks(self.handle, C.byref(n)), self.handle)
        return int(n.value)

    def checkpoint(self):
        """The complete state as a host byte array (mdlg_checkpoint_save)."""
        lib = load()
        b = C.c_size_t(0)
        _check(lib.mdlg_checkpoint_bytes(self.handle, C.byref(b)), self.handle)
        blob = np.zeros(int(b.value), dtype=np.uint8)
        _check(lib.mdlg_checkpoint_save(self.handle, blob.ctypes.data_as(C.c_void_p), blob.size),
               self.handle)
        return blob

    def restore(self, blob):
        """Continue from a checkpoint of a system with the same configuration
        (mdlg_checkpoint_load)."""
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(load().mdlg_checkpoint_load(self.handle, blob.ctypes.data_as(C.c_void_p), blob.size),
               self.handle)

    def reset_accumulators(self):
        _check(load().mdlg_reset_accumulators(self.handle), self.handle)

    def get_f(self, per_site=False):
        f = np.zeros(self.Q)
        counts = np.zeros(self.Q, dtype=np.uint64)
        disp = np.zeros(2 * self.dim)
        ns, no, nl = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        fs = np.zeros((self.n_sites, self.Q)) if per_site else None
        ms = np.zeros((self.n_sites, self.nm)) if per_site else None
        _check(load().mdlg_get_f(self.handle, f.ctypes.data_as(C.c_void_p),
                                 fs.ctypes.data_as(C.c_void_p) if per_site else None,
                                 ms.ctypes.data_as(C.c_void_p) if per_site else None,
                                 counts.ctypes.data_as(C.c_void_p), C.byref(ns), C.byref(no),
                                 disp.ctypes.data_as(C.c_void_p), C.byref(nl)), self.handle)
        out = {"f": f, "counts": counts, "n_samples": ns.value, "n_overflow": no.value,
               "disp_sum": disp[: self.dim].copy(), "disp_sq": disp[self.dim:].copy(),
               "n_lattice_steps": nl.value}
        if per_site:
            out["f_site"] = fs
            out["mom_site"] = ms
        return out

    def kinetics(self):
        out = np.zeros((int(self.cfg.n_replicas), self.dim + 1))
        _check(load().mdlg_get_kinetics(self.handle, out.ctypes.data_as(C.c_void_p)), self.handle)
        return out

    def get_state(self):
        n, d = self.n_total, self.dim
        arrs = {"ucell": np.zeros((n, d), dtype=np.int32), "off": np.zeros((n, d), dtype=np.float32),
                "vel": np.zeros((n, d), dtype=np.float32), "acc": np.zeros((n, d), dtype=np.float32),
                "prev_ucell": np.zeros((n, d), dtype=np.int32),
                "prev_off": np.zeros((n, d), dtype=np.float32)}
        p = MdlgParticles(_ip(arrs["ucell"]), _fp(arrs["off"]), _fp(arrs["vel"]), _fp(arrs["acc"]),
                          _ip(arrs["prev_ucell"]), _fp(arrs["prev_off"]))
        _check(load().mdlg_get_state(self.handle, C.byref(p)), self.handle)
        return arrs

    def set_state(self, ucell, off, vel, prev_ucell=None, prev_off=None):
        n, d = self.n_total, self.dim
        u = np.ascontiguousarray(ucell, dtype=np.int32).reshape(n, d)
        o = np.ascontiguousarray(off, dtype=np.float32).reshape(n, d)
        v = np.ascontiguousarray(vel, dtype=np.float32).reshape(n, d)
        pu = None if prev_ucell is None else np.ascontiguousarray(prev_ucell, dtype=np.int32).reshape(n, d)
        po = None if prev_off is None else np.ascontiguousarray(prev_off, dtype=np.float32).reshape(n, d)
        p = MdlgParticles(_ip(u), _fp(o), _fp(v), None, _ip(pu) if pu is not None else None,
                          _fp(po) if po is not None else None)
        _check(load().mdlg_set_state(self.handle, C.byref(p)), self.handle)
