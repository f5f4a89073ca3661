"""Throughput of the MDLG hot path on one MI355X: particle-steps/s of LJ MD
fused with MDLG binning, for the batched replica ensemble (the default) and
its plain one-system-per-replica counterpart, or for one large system.

One bench step is one lattice time step: md_steps_per_lattice_step MD steps
(forces + velocity Verlet + periodic wrap + cell-list rebuilds) followed by
the binning of every particle (eq. MDni) and the per-site accumulation.
value = particles x MD steps / wall time over the timed lattice steps, with
the state resident in HBM.  Inputs are seeded and synthetic (the paper's own
MD trajectories are not available); see the workload table below.

The JSON line also carries the roofline of the dominant kernel (its
kernel-only time per launch measured with HIP events inside this run), every
kernel class against its own bound, and the FP64 oracle timed on the host
cores (one thread and all threads).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "particle-steps/s (LJ MD + MDLG binning), batched vs plain; % of HBM/FP32 roofline"

# Workloads: seeded synthetic stand-ins for the paper's LAMMPS runs, with
# their sizes, densities, temperatures and lattice steps.
WORKLOADS = {
    "batched": dict(dim=2, n=None, M=None, dx=4.0, kT=1.0, dt=0.005, steps=20, vmax=3,
                    replicas=512,
                    desc="512 2D LJ replicas, N_r log-uniform in [1024, 65536] (seed 4; N_r = 8 M_r^2, "
                         "8,251,320 particles), rho=0.5, kT=1, dt=0.005, 4 sigma lattice per replica, "
                         "Delta t=20 MD steps, V=3 (Q=49); batched (one launch per kernel for all "
                         "replicas) vs plain (one system per replica, launched one after another)"),
    "2d_scale": dict(dim=2, n=262144, M=181, dx=4.0, kT=1.0, dt=0.005, steps=20, vmax=3,
                     desc="2D LJ N=262144, 724 sigma box (rho=0.5), kT=1, dt=0.005, "
                          "181x181 lattice of 4 sigma, Delta t=20 MD steps, V=3 (Q=49)"),
    "2d_small": dict(dim=2, n=2048, M=16, dx=4.0, kT=1.0, dt=0.005, steps=20, vmax=3,
                     desc="2D LJ N=2048, 64 sigma box (rho=0.5), kT=1, dt=0.005, "
                          "16x16 lattice of 4 sigma, Delta t=20 MD steps, V=3 (Q=49)"),
    "3d": dict(dim=3, n=4194304, M=48, dx=4.0, kT=1.5, dt=0.004, steps=20, vmax=2,
               desc="3D LJ N=4194304, 192 sigma cube (rho=0.593), kT=1.5, dt=0.004, "
                    "48^3 lattice of 4 sigma, Delta t=20 MD steps, V=2 (Q=125)"),
    "e1": dict(dim=2, n=100000, M=10, dx=100.0, kT=50.0, dt=1e-4, steps=341600, vmax=3,
               desc="2D hot dilute LJ gas N=100000, 1000 sigma box (rho=0.1), kT=50, dt=1e-4, "
                    "10x10 lattice of 100 sigma, Delta t=341600 MD steps (34.16 tau), V=3 (Q=49), "
                    "plus lattices drifting at u_x = -/+0.05 for theta_3"),
}

# the adjoint of one MD window (gradients of the displacement moments): not a
# lattice-step workload; bench_adjoint times it against the forward window
ADJOINT = dict(dim=2, n=65536, M=90, dx=362.04 / 90, kT=1.0, dt=0.005, vmax=3, window=20, ckpt=5,
               seed=5, desc="2D LJ N=65536, 362.04 sigma box (rho=0.5), kT=1, dt=0.005: adjoint of "
                            "one window of W=20 velocity-Verlet steps, checkpoints every 5 steps, "
                            "loss = per-axis mean squared displacement")

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector, published (256 CUs x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E, published
FLOP_PER_PAIR = {2: 18, 3: 23}  # interacting pair: differences, r^2, rcp, LJ factor, accumulate


def pairs_per_particle(dim, rho, rc=2.5):
    """Ordered neighbours inside r_c at uniform density (the force kernel's
    useful work per particle per step)."""
    return math.pi * rc * rc * rho if dim == 2 else 4.0 / 3.0 * math.pi * rc ** 3 * rho


def force_bytes_per_particle(dim, rho=None, rl=None):
    """HBM bytes per particle of one force/velocity-Verlet step, reported
    beside the FP32 bound: read and write offset and velocity; on the
    pair-list path (list radius rl) also the list, 2 bytes per neighbour
    within rl at uniform density."""
    base = 16 * dim
    if rl is None:
        return base
    vol = math.pi * rl * rl if dim == 2 else 4.0 / 3.0 * math.pi * rl ** 3
    return base + 2 * vol * rho


# FLOPs per interacting pair of the adjoint's reverse step: the force term
# (as FLOP_PER_PAIR), its sigma derivative and the Hessian-vector product
# K (lam_i - lam_j) of the pair
ADJ_FLOP_PER_PAIR = {2: 44, 3: 59}


def adjoint_bytes_per_particle(dim):
    """HBM bytes per particle of one reverse step: read the position and the
    adjoint velocity, read and write the adjoint position, write the new
    adjoint velocity."""
    return 4 * dim * 5


def count_bytes_per_particle(dim):
    """HBM bytes per particle of the counting pass of a cell-list rebuild:
    read offset, image and cell; write the key/slot word."""
    return 4 * dim * 2 + 4 + 8


def scatter_bytes_per_particle(dim):
    """HBM bytes per particle of the permutation pass: read the key/slot
    word, offset, image, cell, velocity, id and the lattice snapshot
    (unwrapped cell, offset); write all of it at the new slot."""
    reads = 8 + 4 * dim * 2 + 4 + 4 * dim + 4 + 8 * dim
    writes = 4 * dim * 3 + 8 + 8 * dim
    return reads + writes


def scan_bytes_per_cell():
    """Read and clear the count, write the cell start."""
    return 12


def sort_bytes(dim, n, cells):
    """Algorithmic bytes of one cell-list rebuild as a unit: keys written and
    read (2 x 4 B) and the payload read and written (2P) per particle, with
    P = offset + cell + velocity + image + id and the permuted lattice
    snapshot (unwrapped cell, offset): 48 B in 2D, 68 B in 3D; 12 B per cell."""
    payload = 48 if dim == 2 else 68
    return n * (8 + 2 * payload) + 12 * cells


def bin_bytes_per_particle(dim, q, nm, per_site_particles):
    """Algorithmic bytes per particle of one binning pass: read offset, image
    and cell, read and write the lattice snapshot (unwrapped cell and offset);
    per site one read-modify-write of the Q counters and the moment
    accumulators, shared by the particles of the site."""
    per_particle = 4 * dim * 2 + 4 + 2 * (8 * dim)
    per_site = 2 * 4 * q + 2 * 8 * nm
    return per_particle + per_site / per_site_particles


def source_digest():
    """Digest of the kernel sources with comments and blank space removed, so
    that a stored counter summary stays valid across comment edits."""
    import re
    h = hashlib.sha256()
    for f in ("mdlg_kernels.hip", "mdlg_force_block.inc", "mdlg_args.h", "mdlg_device.h"):
        with open(os.path.join(ROOT, "paper_1705_04368_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


def _counter_means(folder, counter):
    """Mean value of one rocprofv3 counter per dispatch, by kernel name."""
    import csv
    import glob
    tot = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                name = row["Kernel_Name"]
                name = name.split("(")[0].split("<")[0].replace("void ", "").strip()
                name = name.split("::")[-1]
                s, c = tot.get(name, (0.0, 0))
                tot[name] = (s + float(row["Counter_Value"]), c + 1)
    return {k: s / c for k, (s, c) in tot.items()}


def summarize_traffic(workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, out_dir=None):
    """HBM bytes per launch of each kernel: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled by what the same counters read for a plain copy of 1 GiB.
    Written to <out_dir>/traffic_<workload>.json (default: profiles/)."""
    copy_bytes = float(1 << 30)
    cf = max(_counter_means(copy_fetch_dir, "FETCH_SIZE").values())
    cw = max(_counter_means(copy_write_dir, "WRITE_SIZE").values())
    f_fac, w_fac = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    names = {"k_force": "force", "k_count": "count", "k_scan": "scan", "k_scatter": "scatter",
             "k_bin": "bin", "k_kin": "kin", "k_ingest": "ingest", "k_nlist_narrow": "nlist",
             "k_nlist_wide": "nlist"}
    kernels = {}
    for kname, cls in names.items():
        if kname in fetch and kname in write:
            kernels[cls] = {"fetch_kib": fetch[kname], "write_kib": write[kname],
                            "bytes_per_launch": fetch[kname] * 1024.0 * f_fac
                            + write[kname] * 1024.0 * w_fac}
    out = {"workload": workload, "source_digest": source_digest(),
           "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw,
                                "fetch_factor": f_fac, "write_factor": w_fac},
           "kernels": kernels}
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))
    return out


E1_DU = 0.05  # drift of the two extra lattices of the e1 workload (lattice units per step)


def e1_analysis(sysg, w):
    """The paper-regime analysis of the hot dilute gas from the timed run's
    readouts: a^2 from the measured per-axis mean squared displacement,
    eq. (eqn:Psi), eq. (eqn:Phi), eq. (tet2), eq. (tet3) (lattices drifting at
    u_x = -/+E1_DU), the discrete m_2, all on the full and the one-shell
    velocity set; then the velocity autocorrelation over 1 tau of plain MD
    steps, its exponential fit, eq. (vca) against the measured displacement,
    the a^2 matching the D2Q9 weights and the Delta t(Delta x) of eq. (vca)."""
    from paper_1705_04368_amd import analysis as an
    dim, n = w["dim"], w["n"]
    f = sysg.get_f()
    T = f["n_lattice_steps"]
    msd = f["disp_sq"] / (n * T)
    a2 = float(np.mean(msd)) / w["dx"] ** 2
    fi = f["f"]
    sh = sysg.get_shifts()
    q = len(fi)
    fm, fp = sh["counts"][0][:q].astype(np.float64), sh["counts"][1][:q].astype(np.float64)
    out = {"lattice_steps": T, "a2": a2, "msd_axis": [float(x) for x in msd],
           "mean_velocity": [float(x) for x in (an.lattice_velocities(q, dim).T @ fi) / fi.sum()]}
    for name, g, gm, gp in (("full", fi, fm, fp),
                            ("one_shell", an.one_shell(fi, dim), an.one_shell(fm, dim),
                             an.one_shell(fp, dim))):
        out[name] = {"psi": an.psi(g, dim, a2).tolist(), "phi_xxx": an.phi_xxx(g, dim, a2),
                     "theta2": an.theta2(g, dim, a2), "theta3": an.theta3(gm, gp, E1_DU, dim),
                     "m2_minus_a2": an.m2(g, dim) - a2}
    out["m2_closed_form_minus_a2"] = an.m2(an.equilibrium(dim, 12, a2), dim) - a2
    out["f_minus_closed_form_max"] = float(np.max(np.abs(fi / fi.sum() - an.equilibrium(dim, w["vmax"], a2))))
    # velocity autocorrelation over 1 tau of plain MD steps after the run
    every = 250
    t_steps, c = an.vacf_series(sysg, 40, every)
    t = t_steps * w["dt"]
    early = (t > 0) & (t <= 0.5)
    tau = an.fit_tau(t[early], c[early], w["kT"])
    out["vacf"] = {"t": t.tolist(), "c": c.tolist(), "tau_fit": tau}
    dt_lat = w["steps"] * w["dt"]
    out["msd_eq_vca"] = float(an.msd_exponential(w["kT"], tau, dt_lat))
    out["d2q9_a2"] = {k: an.a2_for_weight(v, wt) for k, (v, wt) in an.D2Q9_WEIGHTS.items()}
    out["dt_for_dx_100_a2_1_6"] = an.dt_for_dx(w["dx"], 1.0 / 6.0, w["kT"], tau)
    return out


def host_cpu():
    """Host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def _oracle_lattice_step(task):
    """One lattice step of the FP64 oracle on one system: Delta t MD steps and
    the binning (the state's forces are evaluated when it is built)."""
    st, lat, steps = task
    st.mdlg(lat, steps, 1)


def cpu_baseline_single(w, x, v, box, M, lattice_steps, budget_s=15.0):
    """The FP64 oracle, one thread, on the full system from the given
    (warmed-up) state, or for more than 300k particles on a smaller periodic
    system of the same density and temperature: MD steps timed one at a time
    until about budget_s seconds (at most lattice_steps lattice steps' worth),
    then one binning pass; the rate is particle-steps per second of that
    work."""
    import oracle
    dim, n = w["dim"], x.shape[0]
    model, _ = host_cpu()
    what = "full system from the warmed-up state"
    if n > 300000:
        # one full-system step of the oracle takes about a minute here: a
        # smaller periodic system of the same density and temperature (a whole
        # number of lattice cells, about 300k particles, synthetic start)
        import synth
        Ms = max(2, int(round(M * (300000.0 / n) ** (1.0 / dim))))
        box = Ms * w["dx"]
        n = int(round(n * (Ms / M) ** dim))
        xs, vs = synth.lj_initial_state(dim, n, box, w["kT"], seed=17)
        x, v, M = xs.astype(np.float64), vs.astype(np.float64), Ms
        what = (f"a {n}-particle system of the same density and temperature ({Ms}^{dim} lattice "
                f"cells, synthetic start)")
        print(f"# cpu baseline: {what}", file=sys.stderr, flush=True)
    md = oracle.make_md(dim, n, box, dt=w["dt"])
    st = oracle.OracleState(md, x, v)
    lat = oracle.make_lattice(dim, (M,) * dim, w["dx"], w["vmax"])
    t0 = time.perf_counter()
    steps = 0
    while steps < lattice_steps * w["steps"] - 1 and time.perf_counter() - t0 < budget_s:
        st.run(1)
        steps += 1
        print(f"# cpu baseline: {steps} MD steps, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    st.mdlg(lat, 1, 1)  # one more MD step and the binning
    steps += 1
    t = time.perf_counter() - t0
    return {"value": n * steps / t, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle", "cpu": model,
            "sample": f"{what}, {steps} MD steps and one binning pass, FP64, one thread, "
                      f"{t:.1f} s"}


def cpu_baseline_ensemble(w, xs, vs, m_r, single_target=400000, threads=None):
    """The FP64 oracle on replicas of the ensemble from the warmed-up state,
    one lattice step (Delta t MD steps + binning) each: on one thread over a
    seeded subset of about `single_target` particles, and on every host core
    available (one replica per task, a thread pool: the oracle's C calls run
    outside the interpreter lock) over all replicas."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    model, avail = host_cpu()
    cores = threads or min(16, avail)
    dim, steps = w["dim"], w["steps"]

    def build(r):
        m = int(m_r[r])
        md = oracle.make_md(dim, xs[r].shape[0], w["dx"] * m, dt=w["dt"])
        return (oracle.OracleState(md, xs[r], vs[r]),
                oracle.make_lattice(dim, (m,) * dim, w["dx"], w["vmax"]), steps)

    order = np.random.default_rng(7).permutation(len(xs))
    sub, tot = [], 0
    for r in order:
        if tot >= single_target:
            break
        sub.append(int(r))
        tot += xs[r].shape[0]
    tasks = [build(r) for r in sub]
    t0 = time.perf_counter()
    for t in tasks:
        _oracle_lattice_step(t)
    t1 = time.perf_counter() - t0
    single = {"value": tot * steps / t1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
              "cpu": model,
              "sample": f"{len(sub)} replicas (seeded subset, {tot} particles), one lattice step "
                        f"each ({steps} MD steps + binning), FP64, one thread, {t1:.1f} s"}
    with ThreadPoolExecutor(max_workers=cores) as ex:
        # largest replicas first for balance
        big = sorted(range(len(xs)), key=lambda r: -xs[r].shape[0])
        tasks = list(ex.map(build, big))
        ntot = sum(xs[r].shape[0] for r in big)
        t0 = time.perf_counter()
        list(ex.map(_oracle_lattice_step, tasks))
        t2 = time.perf_counter() - t0
    return {"value": ntot * steps / t2, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "cpu": model, "cores_available": avail,
            "sample": f"all {len(xs)} replicas ({ntot} particles), one lattice step each ({steps} MD "
                      f"steps + binning), FP64, {cores} threads, {t2:.1f} s",
            "single_thread": single}


def equilibrated_state(sysg, cfg):
    """Positions in [0, box) and velocities of a system, in particle order
    (host float32), to start another system from about the same state (the
    float32 absolute position rounds the offset inside the cell)."""
    st = sysg.get_state()
    s = sysg.layout["cell_side"]
    k = sysg.layout["md_cell_split"]
    n = np.ctypeslib.as_array(cfg.n_particles, shape=(cfg.n_replicas,))
    lat = np.ctypeslib.as_array(cfg.lattice, shape=(cfg.n_replicas * cfg.dim,)).reshape(-1, cfg.dim)
    mc = np.repeat(lat * k, n, axis=0)
    x = np.mod(st["ucell"], mc).astype(np.float64) * s + st["off"].astype(np.float64)
    x32 = x.astype(np.float32)
    box = (mc * s).astype(np.float32)
    x32 = np.where(x32 >= box, np.float32(0.0), x32)
    return np.ascontiguousarray(x32), np.ascontiguousarray(st["vel"].astype(np.float32))


def replica_fi(f_site, m_r):
    """Per replica, f_i = mean n_i per site and lattice step, from the per-site
    time averages; and the replicas' site counts."""
    sites = m_r.astype(np.int64) ** 2
    off = np.concatenate([[0], np.cumsum(sites)[:-1]])
    return np.add.reduceat(f_site, off, axis=0) / sites[:, None], sites


def ensemble_mean_se(fr, w):
    """Site-weighted mean of the replicas' f_i (the ensemble f_i of eq. fieq)
    and its standard error from the spread of the replicas."""
    W = float(w.sum())
    mean = (w[:, None] * fr).sum(axis=0) / W
    R = len(w)
    var = (w[:, None] ** 2 * (fr - mean) ** 2).sum(axis=0) / W ** 2 * R / (R - 1)
    return mean, np.sqrt(var)


def compare_fi(fa, sea, fb, seb, counts_min):
    """z of every bin whose expected count is at least 100 in both runs; the
    Sidak-adjusted 1% threshold over those bins."""
    from scipy.stats import norm
    tested = (counts_min >= 100) & ((sea > 0) | (seb > 0))
    z = (fa - fb)[tested] / np.sqrt(sea[tested] ** 2 + seb[tested] ** 2)
    m = int(tested.sum())
    thr = float(norm.isf((1 - 0.99 ** (1.0 / max(m, 1))) / 2))
    return {"bins_tested": m, "max_abs_z": float(np.abs(z).max()) if m else 0.0,
            "within_3se": int((np.abs(z) <= 3).sum()), "sidak_threshold": thr,
            "agree": bool(m > 0 and np.abs(z).max() < thr and (np.abs(z) <= 3).mean() >= 0.9)}


def plain_replicas(lay, n_r, m_r, w, dev, state, lattice_steps):
    """The same ensemble as one system per replica, launched one after the
    other (each replica's lattice step is its own graph of launches), with the
    batched run's layout (MD-cell split, rebuild interval, brick, block size),
    from `state` (the batched run's, in particle order, imported exactly).
    Returns the throughput and the per-replica f_i."""
    import torch

    from paper_1705_04368_amd import System, make_config
    systems, blobs = [], []
    off = 0
    s = lay["cell_side"]
    k = lay["md_cell_split"]
    for nr, mr in zip(n_r, m_r):
        nr, mr = int(nr), int(mr)
        c = make_config(2, nr, mr, lattice_dx=w["dx"], dt=w["dt"], md_steps_per_lattice_step=w["steps"],
                        vmax=w["vmax"], kT=w["kT"], md_cell_split=k, sort_every=lay["sort_every"],
                        brick=lay["brick"], block_threads=lay["block_threads"],
                        pair_list=lay["pair_slots"] > 0)
        sl = slice(off, off + nr)
        x = (np.mod(state["ucell"][sl], mr * k).astype(np.float64) * s + state["off"][sl]).astype(np.float32)
        x = np.where(x >= np.float32(mr * k * s), np.float32(0.0), x)
        r = System(c, torch.from_numpy(x).to(dev), torch.from_numpy(state["vel"][sl].copy()).to(dev))
        r.set_state(state["ucell"][sl], state["off"][sl], state["vel"][sl])
        blobs.append(r.checkpoint())
        systems.append(r)
        off += nr
    for r, b in zip(systems, blobs):  # capture each replica's graph, then back to the start
        r.coarse_grain(1)
        r.restore(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(lattice_steps):
        for r in systems:
            r.coarse_grain(1)
    for r in systems:
        r.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = int(np.sum(n_r))
    fr = np.stack([r.get_f()["counts"].astype(np.float64) for r in systems])
    fr /= lattice_steps * (m_r.astype(np.float64) ** 2)[:, None]
    for r in systems:
        r.close()
    return {"value": n * lattice_steps * w["steps"] / el, "unit": "particle-steps/s",
            "lattice_steps": lattice_steps, "ms_per_step": el / lattice_steps * 1e3,
            "layout": "the batched run's"}, fr


# rocprofv3 reads the 20 us clock wait of mdlg_timing_offset as 20.60 us: the
# dispatch of a kernel adds 0.6 us that its own duration includes, so that
# much of the clock wait's excess over its span is not the event pair's
CLOCK_WAIT_DISPATCH_MS = 0.0006


def event_pair_offset(sysg):
    """What an event pair adds to a kernel's time, in ms (mdlg_timing_offset
    less the dispatch time of the clock wait itself)."""
    return max(sysg.timing_offset() - CLOCK_WAIT_DISPATCH_MS, 0.0)


def kernel_table(tim, dim, n, rho, lay, n_sites, offset_ms=0.0):
    """Per kernel class: the kernel-only time per launch (HIP events recorded
    around each kernel by its launch, less offset_ms, the constant an event
    pair adds, measured on a kernel of known length (event_pair_offset);
    `event_ms` keeps the raw event average) and the kernel against its own bound:
    the force kernel (and the adjoint's reverse step) on the FP32 vector
    units, with the FLOPs of the interacting pairs; the rebuild passes, the
    pair-list builder and the binning on HBM, with their algorithmic bytes."""
    q, nm = lay["n_velocities"], lay["n_moments"]
    per_site = n / n_sites
    kernels = {}

    def alu(flops, avg):
        tf = flops / (avg * 1e-3) / 1e12
        return {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / PEAK_FP32_TFLOPS, "work_per_launch": flops}

    def hbm(nbytes, avg):
        gb = nbytes / (avg * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gb, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gb / PEAK_HBM_GBS, "work_per_launch": nbytes}

    for k, (ms, cnt) in tim.items():
        if cnt == 0:
            continue
        raw = ms / cnt
        # (an average at or below the offset is left as measured)
        avg = raw - offset_ms if raw > offset_ms else raw
        e = {"avg_ms": avg, "event_ms": raw, "launches": cnt}
        if k == "force":
            e.update(alu(n * pairs_per_particle(dim, rho) * FLOP_PER_PAIR[dim], avg))
            rl = 2.5 + 2 * lay["skin"] if lay["pair_slots"] > 0 else None
            hb = n * force_bytes_per_particle(dim, rho, rl)
            e["hbm_bytes_per_launch"] = hb
            e["hbm_GBs"] = hb / (avg * 1e-3) / 1e9
        elif k == "count":
            e.update(hbm(n * count_bytes_per_particle(dim), avg))
        elif k == "scatter":
            e.update(hbm(n * scatter_bytes_per_particle(dim), avg))
        elif k == "scan":
            e.update(hbm(scan_bytes_per_cell() * lay["n_cells"], avg))
        elif k == "nlist":
            # read the offsets, write the lists (16-bit entries within
            # r_cut + 2 skin) and the target records
            rl = 2.5 + 2 * lay["skin"]
            vol = math.pi * rl * rl if dim == 2 else 4.0 / 3.0 * math.pi * rl ** 3
            e.update(hbm(n * (4 * dim + 2 * vol * rho + 8), avg))
        elif k == "shift":
            e.update(hbm(n * (4 + 16 * dim), avg))
        elif k == "xi":
            e.update(hbm(n_sites * q * (4 + 4 + 16 + 4), avg))
        elif k == "bin":
            e.update(hbm(n * bin_bytes_per_particle(dim, q, nm, per_site), avg))
        elif k == "adjoint":
            e.update(alu(n * pairs_per_particle(dim, rho) * ADJ_FLOP_PER_PAIR[dim], avg))
        elif k == "adjoint_force":
            # a reverse step and a recomputed force step in one launch
            e.update(alu(n * pairs_per_particle(dim, rho) * (ADJ_FLOP_PER_PAIR[dim] + FLOP_PER_PAIR[dim]),
                         avg))
        kernels[k] = e
    sort_unit = None
    if all(k in kernels for k in ("count", "scan", "scatter")):
        t = sum(kernels[k]["avg_ms"] for k in ("count", "scan", "scatter"))
        nbytes = sort_bytes(dim, n, lay["n_cells"])
        gb = nbytes / (t * 1e-3) / 1e9
        sort_unit = {"avg_ms": t, "bound": "hbm", "achieved": gb, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gb / PEAK_HBM_GBS, "work_per_launch": nbytes}
    return kernels, sort_unit


def _r6(d):
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in d.items()}


def bench_adjoint(args):
    """The adjoint of one MD window (mdlg_adjoint: forward window with
    checkpoints, then the reverse sweep recomputing each segment) against the
    forward window alone (W plain MD steps), on an equilibrated 2D system."""
    import torch

    import synth
    from paper_1705_04368_amd import System, describe, make_config
    w = ADJOINT
    dim, n, M, W, K = w["dim"], w["n"], w["M"], w["window"], w["ckpt"]
    dev = torch.device("cuda:0")
    cfg = make_config(dim, n, M, lattice_dx=w["dx"], dt=w["dt"], vmax=w["vmax"], thermostat_every=10,
                      kT=w["kT"], adjoint_window=W, adjoint_every=K)
    lay = describe(cfg)
    box = M * lay["md_cell_split"] * lay["cell_side"]
    pos, vel = synth.lj_initial_state(dim, n, box, w["kT"], seed=w["seed"])
    sysg = System(cfg, torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev))
    sysg.step(args.equilibrate)
    sysg.sync()
    if not args.no_autotune:
        # brick, block size and rebuild interval measured on the equilibrated
        # state; the MD-cell split stays (the box is M k s with s = float32(dx / k))
        from paper_1705_04368_amd import autotune
        cfg.md_cell_split = lay["md_cell_split"]
        xe, ve = equilibrated_state(sysg, cfg)
        cfg, _ = autotune(cfg, torch.from_numpy(xe).to(dev), torch.from_numpy(ve).to(dev),
                          md_steps=args.autotune_steps)
        sysg.close()
        sysg = System(cfg, torch.from_numpy(xe).to(dev), torch.from_numpy(ve).to(dev))
    print(f"# workload adjoint: {w['desc']}; layout {sysg.layout}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sysg.adjoint(W, K, "msd", want_v0=True)
        sysg.step(W)
    sysg.sync()
    torch.cuda.synchronize()
    print("# equilibrated and warmed up", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sysg.step(W)
    sysg.sync()
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sysg.adjoint(W, K, "msd", want_v0=True)
    torch.cuda.synchronize()
    adj = (time.perf_counter() - t0) / args.steps
    print(f"# timed {args.steps} windows: forward {fwd * 1e3:.3f} ms, gradient {adj * 1e3:.3f} ms",
          file=sys.stderr, flush=True)
    sysg.set_timing(True)
    # a device-side wait lets the host enqueue the call's launches ahead, so
    # that they run back to back and no event pair takes in a launch gap
    sysg.timing_head_start(20000)
    sysg.adjoint(W, K, "msd", want_v0=True)
    tim = sysg.get_timing()
    sysg.set_timing(False)
    offset = event_pair_offset(sysg)
    rho = n / box ** dim
    kernels, _ = kernel_table(tim, dim, n, rho, sysg.layout, 1, offset)
    kernels = {k: v for k, v in kernels.items() if k in ("adjoint", "adjoint_force", "force")}
    kd = kernels["adjoint"]
    roofline = {"kernel": "adjoint", "bound": kd["bound"], "achieved": kd["achieved"],
                "peak": kd["peak"], "unit": kd["unit"], "frac": kd["frac"],
                "traffic": load_traffic("adjoint", "adjoint")}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's FP64 adjoint of the same window on the same state
        import oracle
        print("# cpu baseline (oracle adjoint)", file=sys.stderr, flush=True)
        st = sysg.get_state()
        s = sysg.layout["cell_side"]
        x = np.mod(st["ucell"], M * sysg.layout["md_cell_split"]).astype(np.float64) * s + st["off"]
        md = oracle.make_md(dim, n, box, dt=w["dt"])
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.adjoint(md, x, st["vel"].astype(np.float64), W, "msd")
        tc = time.perf_counter() - t0
        cpu = {"value": n * W * reps / tc, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
               "cpu": host_cpu()[0],
               "sample": f"full system, {reps} windows of W={W} (forward + reverse), FP64 single "
                         f"thread, {tc:.1f} s"}
    out = {
        "metric": "particle-steps/s (adjoint window: forward, recompute and reverse sweep)",
        "value": n * W / adj, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": adj * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["desc"], "windows": args.steps, "window": W, "ckpt_every": K,
                   "md_cell_split": sysg.layout["md_cell_split"], "brick": list(sysg.layout["brick"]),
                   "block_threads": sysg.layout["block_threads"], "autotuned": not args.no_autotune},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "adjoint": {"ms_per_window": adj * 1e3, "forward_ms_per_window": fwd * 1e3,
                    "gradient_over_forward": adj / fwd},
        "kernels": {k: _r6(v) for k, v in kernels.items()},
        "event_offset_ms": round(offset, 6),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed lattice steps")
    ap.add_argument("--warmup", type=int, default=5, help="untimed lattice steps")
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS) + ["adjoint"])
    ap.add_argument("--equilibrate", type=int, default=2000, help="thermostatted MD steps")
    ap.add_argument("--timing-steps", type=int, default=10,
                    help="lattice steps of the event-timed per-kernel pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-lattice-steps", type=int, default=4,
                    help="lattice steps of the oracle on one system (about 12 s at 2d_scale)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the ensemble's oracle baseline (0 = every core available, at most 16)")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="lattice steps timed for the plain (one system per replica) path")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain path of the ensemble")
    ap.add_argument("--sort-every", type=int, default=0, help="rebuild interval (0 = automatic)")
    ap.add_argument("--md-cell-split", type=int, default=0, help="MD cells per lattice cell (0 = auto)")
    ap.add_argument("--brick", type=int, nargs=3, default=(0, 0, 0), help="force brick (0 = auto)")
    ap.add_argument("--block-threads", type=int, default=0, help="threads per force block (0 = auto)")
    ap.add_argument("--no-pair-list", action="store_true",
                    help="walk the neighbour cells at every MD step instead of using pair lists")
    ap.add_argument("--collision-stats", action="store_true",
                    help="also record the collision operator Xi of consecutive lattice steps")
    ap.add_argument("--galilean", type=int, default=0,
                    help="also bin on this many lattices drifting with u_x in [0, 0.5]")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's analytic launch shapes instead of measuring candidates")
    ap.add_argument("--autotune-steps", type=int, default=100, help="MD steps timed per candidate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (scales the HBM "
                         "counters of a profiler to bytes)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                             "COPY_WRITE"),
                    help="write profiles/traffic_<workload>.json from four rocprofv3 --pmc "
                         "output folders: FETCH_SIZE and WRITE_SIZE of this bench, then of "
                         "--copy-calibration")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.workload, *args.summarize_traffic)
        return
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(replicas, or spatial domains of one system, would shard across GPUs)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "adjoint":
        bench_adjoint(args)
        return

    import torch

    import synth
    from paper_1705_04368_amd import System, make_config

    w = WORKLOADS[args.workload]
    dim = w["dim"]
    tuning = dict(sort_every=args.sort_every, pair_list=not args.no_pair_list,
                  md_cell_split=args.md_cell_split, brick=tuple(args.brick),
                  block_threads=args.block_threads, collision_stats=args.collision_stats)
    if args.workload == "e1":
        sh = np.zeros((2, 2, dim))
        sh[0, 1, 0], sh[1, 1, 0] = -E1_DU, E1_DU
        tuning["shifts"] = sh
    if args.galilean:
        # drifting lattices u_x = 0 .. 0.5 (the sweep of the figure on the second moment)
        us = np.linspace(0.0, 0.5, args.galilean)
        sh = np.zeros((args.galilean, 2, dim))
        sh[:, 1, 0] = us
        tuning["shifts"] = sh
    dev = torch.device("cuda:0")
    ensemble = bool(w.get("replicas"))
    if ensemble:
        n_r, m_r = synth.replica_sizes(w["replicas"], seed=4)
        seeds = synth.replica_seeds(w["replicas"], seed=4)
        parts = [synth.lj_initial_state(dim, int(nr), w["dx"] * int(mr), w["kT"], seed=sd)
                 for nr, mr, sd in zip(n_r, m_r, seeds)]
        pos = np.concatenate([p for p, _ in parts])
        vel = np.concatenate([v for _, v in parts])
        n = int(n_r.sum())
        rho = 0.5
        lattice = np.stack([m_r, m_r], axis=1)
        n_sites = int((m_r.astype(np.int64) ** 2).sum())
        cfg = make_config(dim, n_r, lattice, lattice_dx=w["dx"], dt=w["dt"],
                          md_steps_per_lattice_step=w["steps"], vmax=w["vmax"], thermostat_every=10,
                          kT=w["kT"], **tuning)
    else:
        n, M = w["n"], w["M"]
        box = M * w["dx"]
        rho = n / box ** dim
        n_sites = M ** dim
        pos, vel = synth.lj_initial_state(dim, n, box, w["kT"], seed=2 if dim == 2 else 3)
        cfg = make_config(dim, n, M, lattice_dx=w["dx"], dt=w["dt"],
                          md_steps_per_lattice_step=w["steps"], vmax=w["vmax"], thermostat_every=10,
                          kT=w["kT"], **tuning)
    sysg = System(cfg, torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev))
    print(f"# workload {args.workload}: {w['desc']}; layout {sysg.layout}", file=sys.stderr, flush=True)
    sysg.step(args.equilibrate)
    sysg.sync()
    print("# equilibrated", file=sys.stderr, flush=True)
    tuned_ms = None
    if not args.no_autotune:
        # launch shapes measured on the equilibrated state (untimed)
        from paper_1705_04368_amd import autotune
        xe, ve = equilibrated_state(sysg, cfg)
        xe, ve = torch.from_numpy(xe).to(dev), torch.from_numpy(ve).to(dev)
        t0 = time.perf_counter()
        cfg, tuned_ms = autotune(cfg, xe, ve, md_steps=args.autotune_steps)
        print(f"# autotuned in {time.perf_counter() - t0:.1f} s: {tuned_ms * 1e3:.2f} us per MD step",
              file=sys.stderr, flush=True)
        sysg.close()
        sysg = System(cfg, xe, ve)
    lay = sysg.layout
    print(f"# timed layout {lay}", file=sys.stderr, flush=True)
    sysg.coarse_grain(args.warmup)
    sysg.sync()
    sysg.reset_accumulators()
    # the state the timed run starts from (the plain path and the oracle
    # start from it too); reading it does not perturb the trajectory
    start = sysg.get_state()
    print(f"# warmed up ({args.warmup} lattice steps)", file=sys.stderr, flush=True)

    # the K timed lattice steps run as five consecutive chunks with HIP events
    # between them on the system's stream (no host synchronisation inside the
    # timed region): the chunks give repeat rates, whose median is reported
    # beside the whole-run value
    nch = min(5, args.steps)
    sizes = [args.steps // nch + (1 if i < args.steps % nch else 0) for i in range(nch)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nch + 1)]
    fallbacks0 = sysg.list_fallbacks()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(sysg.stream)
    for i, k in enumerate(sizes):
        sysg.coarse_grain(k)
        evs[i + 1].record(sysg.stream)
    sysg.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    md_steps = args.steps * w["steps"]
    value = n * md_steps / elapsed
    chunk_values = [n * k * w["steps"] / (evs[i].elapsed_time(evs[i + 1]) * 1e-3)
                    for i, k in enumerate(sizes)]
    repeats = {"chunks": nch, "lattice_steps": sizes, "values": chunk_values,
               "median": float(np.median(chunk_values))}
    print(f"# timed {args.steps} lattice steps in {elapsed:.4f} s", file=sys.stderr, flush=True)
    fallbacks = sysg.list_fallbacks() - fallbacks0
    f = sysg.get_f(per_site=ensemble)
    assert f["counts"].sum() + f["n_overflow"] == n * f["n_lattice_steps"]

    # kernel-only times per launch over a separate pass of the same lattice steps
    sysg.set_timing(True)
    # a device-side wait lets the host enqueue the pass ahead, so that its
    # kernels run back to back and no event pair takes in a launch gap
    sysg.timing_head_start(50000)
    sysg.coarse_grain(args.timing_steps)
    tim = sysg.get_timing()
    sysg.set_timing(False)
    offset = event_pair_offset(sysg)
    print(f"# event-timed {args.timing_steps} lattice steps (event pair offset {offset * 1e3:.2f} us)",
          file=sys.stderr, flush=True)
    kernels, sort_unit = kernel_table(tim, dim, n, rho, lay, n_sites, offset)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    kd = kernels[dom]
    roofline = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["frac"], "traffic": load_traffic(args.workload, dom)}
    if roofline["traffic"] is not None:
        # the counted HBM bytes per launch over the launch's time, beside the
        # graded bound
        gbs = roofline["traffic"] / (kd["avg_ms"] * 1e-3) / 1e9
        roofline["traffic_GBs"] = gbs
        roofline["traffic_frac_of_hbm"] = gbs / PEAK_HBM_GBS

    plain = None
    fi = None
    if ensemble:
        fr_b, sites = replica_fi(f["f_site"], m_r)
        fb, seb = ensemble_mean_se(fr_b, sites)
        rho_site = n / n_sites
        fi = {"f_i_over_rho_rest_axis_diag": [float(fb[24] / rho_site), float(fb[25] / rho_site),
                                              float(fb[32] / rho_site)],
              "replicas": int(len(m_r)), "lattice_steps": int(f["n_lattice_steps"])}
        if not args.no_plain:
            print(f"# plain path ({len(m_r)} systems, {args.plain_steps} lattice steps)",
                  file=sys.stderr, flush=True)
            plain, fr_p = plain_replicas(lay, n_r, m_r, w, dev, start, args.plain_steps)
            plain["batched_over_plain"] = value / plain["value"]
            fp, sep = ensemble_mean_se(fr_p, sites)
            cmin = np.minimum(fb * n_sites * f["n_lattice_steps"], fp * n_sites * args.plain_steps)
            plain["f_i_batched_vs_plain"] = compare_fi(fb, seb, fp, sep, cmin)

    cpu = None
    if not args.no_cpu_baseline and args.workload != "e1":
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        s = lay["cell_side"]
        k = lay["md_cell_split"]
        if ensemble:
            mc = np.repeat(lattice * k, n_r, axis=0)
            xw = np.mod(start["ucell"], mc).astype(np.float64) * s + start["off"].astype(np.float64)
            bounds = np.concatenate([[0], np.cumsum(n_r)])
            xs = [xw[bounds[r]:bounds[r + 1]] for r in range(len(n_r))]
            vs = [start["vel"][bounds[r]:bounds[r + 1]].astype(np.float64) for r in range(len(n_r))]
            cpu = cpu_baseline_ensemble(w, xs, vs, m_r, threads=args.cpu_threads or None)
        else:
            xw = np.mod(start["ucell"], w["M"] * k).astype(np.float64) * s + start["off"].astype(np.float64)
            cpu = cpu_baseline_single(w, xw, start["vel"].astype(np.float64), w["M"] * w["dx"], w["M"],
                                      args.cpu_lattice_steps)

    out = {
        "metric": METRIC if ensemble else "particle-steps/s (LJ MD + MDLG binning)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "lattice_steps": args.steps, "md_steps": md_steps,
                   "particles": n, "md_cell_split": lay["md_cell_split"], "sort_every": lay["sort_every"],
                   "brick": list(lay["brick"]), "block_threads": lay["block_threads"],
                   "pair_slots": lay["pair_slots"], "list_skin": lay["skin"],
                   "list_fallback_launches": fallbacks, "autotuned": tuned_ms is not None,
                   "collision_stats": args.collision_stats, "galilean_lattices": args.galilean},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "repeats": repeats,
        "plain": plain,
        "f_i": fi,
        "kernels": {k: _r6(v) for k, v in kernels.items()},
        "event_offset_ms": round(offset, 6),
        "sort": None if sort_unit is None else _r6(sort_unit),
    }
    if args.workload == "e1":
        print("# e1 analysis", file=sys.stderr, flush=True)
        out["analysis"] = e1_analysis(sysg, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
