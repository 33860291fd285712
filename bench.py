"""Benchmark of the free-surface cumulant LBM step on one MI355X.

One step = one pass of the whole hot path (dense stream-collide, interface
stream-collide with normals/curvature, reconstruction and mass flux,
conversion, excess mass, the estimator's geometry) over the large synthetic
sediment flume 3072 x 80 x 256 (62.9 M cells: three layers of diameter-10
spheres, 9,210 of them, with small prescribed velocities, 60 cells of
liquid above the bed, FP32 PDF storage, 2000 steps).  The main form runs the
learned interface estimator with its finite-difference fallback where the
network's gate passes (better than finite differences on held-out stencils
and in the flume's own flow); the plain FP32 form, the FP16-storage form and
the network forced on (timed over 300 steps) run on the same lattice; the
1536 x 40 x 192 flume is a sub-entry (FP32, FP16, FP64, 1000 steps); the
velocity and fill-level errors of each storage form against the FP64 oracle
are measured on a 128 x 40 x 192 flume crop after 500 steps and on the
channel film after 200 steps.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32-learned]

HBM traffic of the dense kernel comes from two rocprofv3 counter runs of
this same command (FETCH_SIZE, then WRITE_SIZE), summarised by

    python bench.py --pmc-summary FETCH_DIR WRITE_DIR > profiles/<name>.md

The 1 GiB device copy that the bench times (rocclr copyBuffer) calibrates
the counters; the summary stores a hash of the dense kernel's sources and
the traffic is reported only while the sources still match.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
COPY_BYTES = 1 << 30          # the calibration copy: 1 GiB read + 1 GiB written
BULK_SOURCES = ["paper_2301_10674_amd/csrc/fsl_step.hip", "paper_2301_10674_amd/csrc/fsl_device.h",
                "paper_2301_10674_amd/csrc/fsl_kernels.h"]
KERNEL_NAMES = {"fp32": "k_bulk<float, false>", "fp64": "k_bulk<double, false>", "fp16": "k_bulkIDF16_Lb0E"}


def bulk_source_hash():
    h = hashlib.sha256()
    for f in BULK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    return [r for f in files for r in csv.DictReader(open(f))]


def counter_means(rows, copy_grid):
    """Mean counter value (KiB per dispatch) of the dense kernel per storage
    form and of the calibration copies (copyBuffer dispatches of grid size
    copy_grid)."""
    vals = {}
    for r in rows:
        name = r["Kernel_Name"]
        key = None
        if "copyBuffer" in name and r["Grid_Size"] == copy_grid:
            key = "copy"
        for prec, kn in KERNEL_NAMES.items():
            if kn in name:
                key = prec
        if key:
            vals.setdefault(key, []).append(float(r["Counter_Value"]))
    return rows[0]["Counter_Name"], {k: sum(v) / len(v) for k, v in vals.items()}, \
        {k: len(v) for k, v in vals.items()}


def pmc_summary(fetch_dir, write_dir):
    rf, rw = counter_rows(fetch_dir), counter_rows(write_dir)
    # the calibration copies are the copyBuffer dispatches that write 1 GiB
    grids = {r["Grid_Size"] for r in rw if "copyBuffer" in r["Kernel_Name"]
             and abs(float(r["Counter_Value"]) * 1024.0 - COPY_BYTES) < 0.01 * COPY_BYTES}
    assert len(grids) == 1, grids
    g = grids.pop()
    cf, fetch, nf = counter_means(rf, g)
    cw, write, nw = counter_means(rw, g)
    assert cf == "FETCH_SIZE" and cw == "WRITE_SIZE", (cf, cw)
    # the copy moves COPY_BYTES each way: scale = true bytes / counted bytes
    kf = COPY_BYTES / (fetch["copy"] * 1024.0)
    kw = COPY_BYTES / (write["copy"] * 1024.0)
    out = {"source_hash": bulk_source_hash(), "fetch_scale": kf, "write_scale": kw, "forms": {}}
    lines = ["| form | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | read GB | written GB | traffic GB |",
             "|---|---:|---:|---:|---:|---:|"]
    for prec in ("fp32", "fp16", "fp64"):
        if prec in fetch and prec in write:
            rd = fetch[prec] * 1024.0 * kf / 1e9
            wr = write[prec] * 1024.0 * kw / 1e9
            out["forms"][prec] = {"fetch_kib": fetch[prec], "write_kib": write[prec], "read_gb": rd,
                                  "write_gb": wr, "traffic_gb": rd + wr, "dispatches": nf[prec]}
            lines.append("| %s | %.0f | %.0f | %.3f | %.3f | %.3f |" % (prec, fetch[prec], write[prec], rd, wr, rd + wr))
    print("Calibration: the 1 GiB device copy reads %.0f KiB (FETCH_SIZE) and writes %.0f KiB "
          "(WRITE_SIZE) per dispatch, so the scales are x%.3f and x%.3f.\n" % (fetch["copy"], write["copy"], kf, kw))
    print("\n".join(lines))
    print("\n```json\n%s\n```" % json.dumps(out, indent=1))


def trace_summary(d):
    """Per-kernel table from a rocprofv3 --kernel-trace --stats run (CSV)."""
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % d)
    rows = list(csv.DictReader(open(files[0])))
    print("| kernel | calls | avg µs | min µs | max µs | total ms | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        name = re.sub(r"\(.*", "", r["Name"].replace("(anonymous namespace)::", "")).replace("void ", "")
        print("| %s | %s | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))


def stored_traffic(workload, precision):
    """Traffic per launch (bytes) of the dense kernel from the committed
    counter summary, or None when there is none or the sources changed."""
    f = os.path.join(ROOT, "profiles", "k_bulk_%s_traffic.md" % workload)
    if not os.path.exists(f):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(f).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != bulk_source_hash() or precision not in d.get("forms", {}):
        return None
    return d["forms"][precision]["traffic_gb"] * 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fluid_counts(lat, fsl):
    t = lat.read(fsl.FIELD_TYPE)
    liq = int((t == fsl.LIQUID).sum())
    itf = int((t == fsl.INTERFACE).sum())
    return liq, itf


def interface_error(lat, fsl):
    """RMS angle (degrees) and RMS curvature error of the normals and
    curvatures the lattice uses, against height-function labels of its own
    fill field (interface cells whose 3x3 columns of 7 cells are bracketed
    by liquid and gas)."""
    from paper_2301_10674_amd import estimator as E
    from paper_2301_10674_amd import train as T

    X, Y, cells = T.lattice_samples(lat, fsl)
    f = lat.read_fields([fsl.FIELD_NORMAL, fsl.FIELD_CURV])
    n = f[fsl.FIELD_NORMAL].reshape(3, -1)[:, cells].T
    k = f[fsl.FIELD_CURV].reshape(-1)[cells]
    ang, kap = E.errors(np.concatenate([n, k[:, None]], axis=1), Y)
    return {"rms_angle_deg": ang, "rms_kappa": kap, "cells": int(len(cells))}


def learned_weights(lat, fsl, n_analytic=1000000, ss=16, n_flume=200000, steps=200, every=50, epochs=30,
                    seed=0):
    """Train the estimator: n_analytic analytic stencils (fill levels
    supersampled on ss^3 points per cell on the GPU) plus height-function
    labelled stencils of the lattice's own fill fields (taken while it runs
    the plain estimator); returns weights and report."""
    from paper_2301_10674_amd import train as T

    t0 = time.perf_counter()
    Xa, Ya = T.analytic_dataset_gpu(fsl, n_analytic, seed=seed, ss=ss)
    Xf, Yf = T.flume_dataset(lat, fsl, steps, every, n_flume, seed=seed)
    X, Y = np.concatenate([Xa, Xf]), np.concatenate([Ya, Yf])
    Xt, Yt, Xv, Yv = T.split(X, Y, 0.1, seed=seed)
    rep = T.train(fsl, Xt, Yt, Xv, Yv, epochs=epochs, seed=seed)
    rep["data_seconds"] = time.perf_counter() - t0 - rep["train_seconds"]
    rep.update(analytic_samples=int(len(Xa)), flume_samples=int(len(Xf)), epochs=epochs,
               supersampling="%d^3 points per cell (GPU)" % ss)
    w = rep.pop("weights")
    rep.pop("losses")
    return w, rep


def droplet_check(fsl, weights, steps=2000, R=10.0, n=40, sigma=1e-3):
    """A static droplet (radius R in an n^3 box, sigma, no gravity, FP32) with
    finite differences and with the network: the Laplace jump of the core
    density against 6 sigma / R (Section 2.1's 2 sigma kappa) and the
    largest speed left (spurious currents)."""
    from paper_2301_10674_amd import inputs

    w = inputs.droplet(n=n, radius=R, sigma=sigma)
    x = np.arange(n) + 0.5 - 0.5 * n
    r = np.sqrt(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)
    out = {"steps": steps, "radius": R, "sigma": sigma}
    for name, wts in (("finite_differences", None), ("network", weights)):
        lat = fsl.lattice_from_workload(w, "fp32", normals=1 if wts is not None else 0, check_every=50)
        if wts is not None:
            lat.set_estimator(wts)
        try:
            lat.step(steps)
            f = lat.read_fields([fsl.FIELD_TYPE, fsl.FIELD_RHO, fsl.FIELD_VEL])
            t = f[fsl.FIELD_TYPE]
            core = (t == fsl.LIQUID) & (r < R - 3)
            fluid = (t == fsl.LIQUID) | (t == fsl.INTERFACE)
            drho = float(f[fsl.FIELD_RHO][core].mean() - 1.0)
            out[name] = {"laplace_rel_err": drho / (6.0 * sigma / R) - 1.0,
                         "max_speed": float(np.sqrt((f[fsl.FIELD_VEL][:, fluid] ** 2).sum(0)).max())}
        except fsl.FslError as e:
            out[name] = {"unstable": str(e)}
        lat.destroy()
    return out


def flow_check(w, fsl, weights, steps=1000, check_every=10):
    """The network in the flow it serves: the lattice runs `steps` steps with
    the network and with finite differences alone (watchdog on); the network
    passes if its run stays healthy and its normals and curvatures are at
    least as close to the height-function labels of its own fill field as
    the finite-difference ones are to theirs."""
    out = {"steps": steps}
    for name, wts in (("network", weights), ("finite_differences", None)):
        lat = fsl.lattice_from_workload(w, "fp32", normals=1 if wts is not None else 0,
                                        check_every=check_every)
        if wts is not None:
            lat.set_estimator(wts)
        try:
            lat.step(steps)
            out[name] = interface_error(lat, fsl)
        except fsl.FslError as e:
            out[name] = {"unstable": str(e)}
        lat.destroy()
    net, fd = out["network"], out["finite_differences"]
    out["pass"] = bool("unstable" not in net and "unstable" not in fd
                       and net["rms_angle_deg"] <= fd["rms_angle_deg"] and net["rms_kappa"] <= fd["rms_kappa"])
    return out


def time_particles(w, fsl, precision, steps=20, coupled_steps=20):
    """Particle motion on the flume's spheres (lowest layer fixed, 10
    sub-steps per lattice step, the paper's collision parameters, gravity
    of the flume, lubrication below 2/3 cell) under the lattice's
    momentum-exchange load, then whole coupled steps (fluid step, forces,
    particle sub-steps, remap).  The generated bed is a jittered packing
    whose spheres overlap, so it is first relaxed without fluid (restitution
    0.1, gravity 1e-3, 300 steps) and the lattice is built on the relaxed
    bed."""
    import dataclasses

    import torch

    from paper_2301_10674_amd.couple import Coupled

    c, r = w.centre, w.radius
    fixed = (c[:, 2] < c[:, 2].min() + 2.0).astype(np.uint8)
    nu = (1.0 / w.omega - 0.5) / 3.0
    out = {"spheres": int(len(r)), "fixed": int(fixed.sum()), "substeps": 10}
    try:
        relax = fsl.Dem(w.shape, c, r, None, None, fixed, restitution=0.1, friction=0.5,
                        accel=(0.0, 0.0, -1e-3), substeps=10, skin=1.0)
        relax.step(None, n=300)
        c2, v2, _ = relax.state()
        relax.destroy()
        out["relaxed_max_speed"] = float(np.abs(v2).max())
        wr = dataclasses.replace(w, centre=c2, sphere_vel=np.zeros_like(c2), sphere_angvel=np.zeros_like(c2))
        lat = fsl.lattice_from_workload(wr, precision)
        lat.step(5)
        dem = fsl.Dem(w.shape, c2, r, None, None, fixed, viscosity=nu, lub_cut=2.0 / 3.0,
                      accel=w.accel, substeps=10, skin=1.0)
        hydro = lat.particle_forces()
        dem.step(hydro)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dem.step(hydro)
        out["dem_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
        dem.destroy()
        dem = fsl.Dem(w.shape, c2, r, None, None, fixed, viscosity=nu, lub_cut=2.0 / 3.0,
                      accel=w.accel, substeps=10, skin=1.0)
        run = Coupled(lat, dem)
        run.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.step(coupled_steps)
        torch.cuda.synchronize()
        out["coupled_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / coupled_steps
        # the same sequence phase by phase (each phase synchronised)
        ph = np.zeros(4)
        for _ in range(coupled_steps):
            t = [time.perf_counter()]
            lat.step(1)
            torch.cuda.synchronize()
            t.append(time.perf_counter())
            hydro = lat.particle_forces()
            t.append(time.perf_counter())
            dem.step(hydro)
            t.append(time.perf_counter())
            lat.move_particles(*dem.state())
            t.append(time.perf_counter())
            ph += np.diff(t)
        out["coupled_phases_ms"] = dict(zip(("fluid_step", "forces", "particle_substeps", "remap"),
                                            (1e3 * ph / coupled_steps).round(4).tolist()))
        out["bedload_rate"] = dem.bedload()      # Eq. (1) after the coupled steps
        dem.destroy()
        lat.destroy()
    except fsl.FslError as e:
        out["error"] = str(e)
    return out


_WEIGHTS = {}
TRAIN = {"samples": 1000000, "epochs": 30, "checks": True}


def trained_estimator(fsl):
    """Weights of the learned estimator, trained once per run on analytic
    stencils and height-function labelled fields of the 1536 x 40 x 192
    flume (taken while it runs the plain estimator), and its gate: better
    than finite differences on held-out stencils and in the flume's flow."""
    if "w" not in _WEIGHTS:
        from paper_2301_10674_amd import inputs

        w = inputs.flume(seed=2)
        lat = fsl.lattice_from_workload(w, "fp32")
        weights, rep = learned_weights(lat, fsl, n_analytic=TRAIN["samples"], epochs=TRAIN["epochs"])
        lat.destroy()
        rep["held_out_gate"] = rep.pop("gate")
        if TRAIN["checks"]:
            rep["flow_check"] = flow_check(w, fsl, weights)
            rep["droplet"] = droplet_check(fsl, weights)
            rep["gate"] = bool(rep["held_out_gate"] and rep["flow_check"]["pass"])
        else:
            rep["gate"] = False       # not checked in the flow: not used
        _WEIGHTS["w"], _WEIGHTS["report"] = weights, rep
    return _WEIGHTS["w"], dict(_WEIGHTS["report"])


def run_form(w, form, steps, warmup, main_form=None, particles=True):
    import torch

    from paper_2301_10674_amd import fsl

    precision = form.split("-")[0]
    # "-learned": the network where its gate passes; "-learned-forced": the
    # network whatever its gate says (to time it); "-variants": Thuerey's
    # flux modifiers and normal-weighted excess mass, curvature from corner
    # normals
    learned, forced = "-learned" in form, form.endswith("-forced")
    variants = form.endswith("-variants")
    est = None
    if learned:
        weights, est = trained_estimator(fsl)
    on = learned and (forced or est["gate"])
    lat = fsl.lattice_from_workload(w, precision, normals=1 if on else 0,
                                    flux_modifiers=variants, normal_excess=variants, csf_curvature=variants)
    if on:
        lat.set_estimator(weights)
    lat.step(warmup)
    torch.cuda.synchronize()
    liq0, itf0 = fluid_counts(lat, fsl)
    M0 = lat.total_mass()
    used0 = lat.estimator_stats() if on else (0, 0)
    lat.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.timing(False)
    bulk_ms, launches = lat.timing_read()
    # the global mass right after steps (from the last step's partials)
    t0m = time.perf_counter()
    for _ in range(10):
        M1 = lat.total_mass()
    total_mass_us = 1e6 * (time.perf_counter() - t0m) / 10
    liq1, itf1 = fluid_counts(lat, fsl)
    secs = t1 - t0
    liq = 0.5 * (liq0 + liq1)
    fluid = 0.5 * (liq0 + itf0 + liq1 + itf1)
    s = STORE_BYTES[precision]
    bulk_avg_s = bulk_ms / 1e3 / max(launches, 1)
    bytes_per_launch = liq * (54 * s + 16) + w.ncells * 1
    pdf_bytes_per_launch = liq * 54 * s
    # whole step: the dense pass plus the interface cells (own and pulled
    # PDFs read, PDFs written, fill level, mass, density, mark)
    itf = 0.5 * (itf0 + itf1)
    bytes_per_step = bytes_per_launch + itf * (81 * s + 44)
    res = dict(
        form=form, precision=precision, secs=secs, ms_per_step=1e3 * secs / steps,
        mlups_fluid=fluid * steps / secs / 1e6, mlups_all=w.ncells * steps / secs / 1e6,
        bulk_us=1e6 * bulk_avg_s, bulk_launches=launches,
        bulk_gbs=bytes_per_launch / bulk_avg_s / 1e9, bytes_per_launch=bytes_per_launch,
        bulk_pdf_gbs=pdf_bytes_per_launch / bulk_avg_s / 1e9,
        step_gbs=bytes_per_step / (secs / steps) / 1e9, bytes_per_step=bytes_per_step,
        liquid_cells=liq, fluid_cells=fluid, interface_cells=0.5 * (itf0 + itf1),
        mass_drift=abs(M1 - M0) / M0, total_mass_us=total_mass_us, interface_error=interface_error(lat, fsl))
    if learned:
        used1 = lat.estimator_stats() if on else (0, 0)
        res["estimator"] = dict(est, network_on=on, network_cells=used1[0] - used0[0],
                                fallback_cells=used1[1] - used0[1])
    if len(w.radius) and form == main_form and particles:
        res["particles"] = time_particles(w, fsl, precision)
    # momentum-exchange force and torque on every sphere (outside the timed
    # steps; the coupling would call it once per step)
    if len(w.radius):
        lat.particle_forces()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            lat.particle_forces()
        res["particle_forces_ms"] = 1e3 * (time.perf_counter() - t0) / 10
    lat.destroy()
    del lat
    torch.cuda.synchronize()
    return res


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write counted), best of reps."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    return best


def cpu_baseline(ny, nz, seconds_target=12.0):
    """The FP64 oracle on the bench's flume recipe (same ny, nz, seed 3) on
    a 64-cell-long periodic box, for as many steps as fit in about
    seconds_target: once on one thread (the reported value) and once on all
    host threads (its per-cell phases run in parallel; the result does not
    depend on the thread count)."""
    from oracle import oracle as O
    from paper_2301_10674_amd import inputs

    w = inputs.flume(nx=64, ny=ny, nz=nz, seed=3)

    def timed(threads):
        used = O.set_threads(threads)
        o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                            conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel)
        o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
        t = o.read(O.F_TYPE)
        fluid = int(((t == O.LIQUID) | (t == O.INTERFACE)).sum())
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        n = max(1, int(seconds_target / max(one, 1e-3)) - 1)
        t0 = time.perf_counter()
        o.step(n)
        secs = time.perf_counter() - t0
        return fluid * n / secs / 1e6, used, fluid, n, secs

    v1, c1, fluid, n1, s1 = timed(1)
    va, ca, _, na, sa = timed(0)
    # the channel film (64 x 8 x 32, 200 steps) on one thread and on all
    wf = inputs.channel_film()
    film = {}
    for threads in (1, 0):
        used = O.set_threads(threads)
        o = O.OracleLattice(wf.shape, wf.omega, accel=wf.accel, sigma=wf.sigma, rho_gas=wf.rho_gas,
                            conv_eps=wf.conv_eps, fill=wf.fill, rho=wf.rho, vel=wf.vel)
        o.set_particles(wf.centre, wf.radius, wf.sphere_vel, wf.sphere_angvel)
        t = o.read(O.F_TYPE)
        nf = int(((t == O.LIQUID) | (t == O.INTERFACE)).sum())
        t0 = time.perf_counter()
        o.step(200)
        film["threads_%d" % used] = nf * 200 / (time.perf_counter() - t0) / 1e6
    O.set_threads(0)
    return {"value": v1, "unit": "MLUPS (fluid cells)", "cores": c1, "kind": "oracle",
            "sample": "FP64 oracle, the flume recipe on a 64x%dx%d periodic box (%d fluid cells), "
                      "%d steps after 1 warm-up step, %.1f s on 1 thread" % (ny, nz, fluid, n1, s1),
            "all_cores": {"value": va, "cores": ca,
                          "sample": "%d steps after 1 warm-up step, %.1f s on %d threads" % (na, sa, ca)},
            "channel_film_64x8x32": dict(film, unit="MLUPS (fluid cells)", sample="200 steps")}


def gpu_weights(w):
    """The estimator weights as the GPU multiplies with them: the three
    matrices rounded to BF16 (nearest, ties to even), biases in FP32."""
    p = np.asarray(w, dtype=np.float64).copy()
    for a, b in ((0, 1728), (1792, 5888), (5952, 6208)):
        u = np.ascontiguousarray(w[a:b], dtype=np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        p[a:b] = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return p


def accuracy_vs_oracle(weights=None, crop_steps=500, film_steps=200, crop5_steps=200):
    """Velocity and fill-level error of each storage form against the FP64
    oracle on the same seeded inputs: the flume recipe on its own periodic
    128 x 40 x 192 box after crop_steps steps (also the oracle's own error
    when it stores FP16 deviations: the floor of any FP16-storage form), the
    large flume's recipe on a 64 x 80 x 256 box after crop5_steps steps, and
    the channel film 64 x 8 x 32 after film_steps steps, where the learned
    form is compared with the oracle running the same (BF16-rounded) network
    with the same fallback rules."""
    from oracle import oracle as O
    from paper_2301_10674_amd import fsl, inputs

    def fluid(t):
        return (t == O.LIQUID) | (t == O.INTERFACE)

    def oracle_run(w, steps, store="fp64", params=None):
        o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                            conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel, store=store)
        o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
        if params is not None:
            o.set_estimator(params)
        M0 = o.total_mass()
        o.step(steps)
        r = {"type": o.read(O.F_TYPE), "vel": o.read(O.F_VEL), "fill": o.read(O.F_FILL),
             "drift": abs(o.total_mass() - M0) / M0}
        del o
        return r

    def compare(tg, vg, fg, ref):
        both = fluid(tg) & fluid(ref["type"])
        d = vg[:, both] - ref["vel"][:, both]
        vel = float(np.sqrt((d ** 2).sum() / (ref["vel"][:, both] ** 2).sum()))
        bi = (tg == O.INTERFACE) & (ref["type"] == O.INTERFACE)
        df = np.abs(fg[bi] - ref["fill"][bi])
        return {"velocity_rel_l2": vel, "fill_max": float(df.max(initial=0.0)),
                "fill_mean": float(df.mean()) if df.size else 0.0,
                "type_mismatches": int((tg != ref["type"]).sum())}

    def gpu_run(w, steps, prec, learned=False):
        g = fsl.lattice_from_workload(w, prec, normals=1 if learned else 0)
        if learned:
            g.set_estimator(weights)
        M0 = g.total_mass()
        g.step(steps)
        f = g.read_fields([fsl.FIELD_TYPE, fsl.FIELD_VEL, fsl.FIELD_FILL])
        drift = abs(g.total_mass() - M0) / M0
        g.destroy()
        return f[fsl.FIELD_TYPE], f[fsl.FIELD_VEL], f[fsl.FIELD_FILL], drift

    O.set_threads(0)
    out = {}
    w = inputs.flume_crop(nx=128, seed=3)
    t0 = time.perf_counter()
    ref = oracle_run(w, crop_steps)
    floor = oracle_run(w, crop_steps, store="fp16")
    crop = {"steps": crop_steps, "oracle_seconds": time.perf_counter() - t0,
            "oracle_fp16_storage": dict(compare(floor["type"], floor["vel"], floor["fill"], ref),
                                        mass_drift=floor["drift"])}
    for prec in ("fp64", "fp32", "fp16"):
        tg, vg, fg, drift = gpu_run(w, crop_steps, prec)
        crop[prec] = dict(compare(tg, vg, fg, ref), mass_drift=drift)
    v16 = crop["fp16"]["velocity_rel_l2"]
    crop["targets"] = {"fp32_velocity_1e-5": crop["fp32"]["velocity_rel_l2"] <= 1e-5,
                       "fp16_velocity_1e-3": v16 <= 1e-3,
                       "fp16_within_1.5x_oracle_fp16_floor":
                           v16 <= 1.5 * crop["oracle_fp16_storage"]["velocity_rel_l2"],
                       "mass_drift_1e-12": max(crop[p]["mass_drift"] for p in ("fp64", "fp32", "fp16")) <= 1e-12}
    out[w.name] = crop
    log("accuracy crop:", json.dumps(crop))

    # the large flume's recipe (80 x 256 cross-section) on a 64-cell-long box
    w = inputs.flume(nx=64, ny=80, nz=256, seed=3)
    ref = oracle_run(w, crop5_steps)
    c5 = {"steps": crop5_steps}
    for prec in ("fp64", "fp32", "fp16"):
        tg, vg, fg, drift = gpu_run(w, crop5_steps, prec)
        c5[prec] = dict(compare(tg, vg, fg, ref), mass_drift=drift)
    out[w.name] = c5
    log("accuracy large-flume crop:", json.dumps(c5))

    w = inputs.channel_film()
    ref = oracle_run(w, film_steps)
    film = {"steps": film_steps}
    for prec in ("fp64", "fp32", "fp16"):
        tg, vg, fg, drift = gpu_run(w, film_steps, prec)
        film[prec] = dict(compare(tg, vg, fg, ref), mass_drift=drift)
    if weights is not None:
        # the oracle runs the network from the same BF16-rounded weights
        ref_l = oracle_run(w, film_steps, params=gpu_weights(weights))
        tg, vg, fg, drift = gpu_run(w, film_steps, "fp64", learned=True)
        film["fp64-learned"] = dict(compare(tg, vg, fg, ref_l), mass_drift=drift)
        film["learned_vs_plain_oracle"] = compare(ref_l["type"], ref_l["vel"], ref_l["fill"], ref)
    out[w.name] = film
    log("accuracy film:", json.dumps(film))
    return out


def dem_only(w, steps=50):
    """Particle steps alone on the flume's spheres (radius 5, lowest layer
    fixed, 10 sub-steps, lubrication below 2/3 cell, skin 1 cell, no
    hydrodynamic load): the command behind the particle kernel trace."""
    import torch

    from paper_2301_10674_amd import fsl

    c, r = w.centre, w.radius
    fixed = (c[:, 2] < c[:, 2].min() + 2.0).astype(np.uint8)
    nu = (1.0 / w.omega - 0.5) / 3.0
    dem = fsl.Dem(w.shape, c, r, None, None, fixed, viscosity=nu, lub_cut=2.0 / 3.0,
                  accel=w.accel, substeps=10, skin=1.0)
    dem.step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dem.step(None)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    dem.destroy()
    print(json.dumps({"workload": w.name, "spheres": int(len(r)), "fixed": int(fixed.sum()),
                      "steps": steps, "substeps": 10, "ms_per_step": ms}), flush=True)


def form_summary(v):
    return {kk: v[kk] for kk in ("mlups_fluid", "ms_per_step", "bulk_us", "bulk_gbs", "mass_drift", "total_mass_us",
                                 "interface_error", "estimator", "particle_forces_ms", "particles",
                                 "steps") if kk in v}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32-learned",
                    choices=["fp32", "fp16", "fp64", "fp32-learned", "fp16-learned", "fp32-learned-forced"])
    ap.add_argument("--nx", type=int, default=3072)
    ap.add_argument("--ny", type=int, default=80)
    ap.add_argument("--nz", type=int, default=256)
    ap.add_argument("--forms", default="fp32,fp16,fp32-learned-forced",
                    help="other forms timed on the same flume ('' for none): fp16, fp64, fp32, "
                         "fp32-learned (estimator trained in the run, see train.py, used where its gate "
                         "passes), fp32-learned-forced (the network on whatever its gate says, timed over "
                         "at most 300 steps), fp32-variants (flux modifiers, normal-weighted excess mass, "
                         "corner-normal curvature)")
    ap.add_argument("--sub", default="1536x40x192:fp32,fp16,fp64",
                    help="a second flume and its forms, NXxNYxNZ:form,form ('' for none)")
    ap.add_argument("--sub-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy runs against the oracle")
    ap.add_argument("--no-particles", action="store_true", help="skip the particle and coupled-step timing")
    ap.add_argument("--train-samples", type=int, default=1000000, help="analytic training stencils")
    ap.add_argument("--train-epochs", type=int, default=30)
    ap.add_argument("--no-estimator-checks", action="store_true",
                    help="skip the estimator's checks in the flume's flow and on the droplet (it is then not used "
                         "except in the -forced form)")
    ap.add_argument("--dem-only", action="store_true",
                    help="time particle steps alone on the flume's spheres and exit")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 counter runs of this command and exit")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run of this command and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2301_10674_amd import fsl, inputs

    TRAIN.update(samples=args.train_samples, epochs=args.train_epochs, checks=not args.no_estimator_checks)
    fsl.lib()  # fails loudly if the HIP library is missing
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    log("building flume %dx%dx%d" % (args.nx, args.ny, args.nz))
    w = inputs.flume(nx=args.nx, ny=args.ny, nz=args.nz, seed=2)
    log("spheres %d, bed height %.2f, surface %.2f" % (w.meta["spheres"], w.meta["bed_height"],
                                                      w.meta["surface"]))
    if args.dem_only:
        dem_only(w)
        return
    meta = dict(w.meta)
    main_res = run_form(w, args.precision, args.steps, args.warmup, main_form=args.precision,
                        particles=not args.no_particles)
    main_res["steps"] = args.steps
    log("main form:", json.dumps(main_res))
    forms = {args.precision: main_res}
    for p in [f for f in args.forms.split(",") if f and f != args.precision]:
        k = min(args.steps, 300) if p.endswith("-forced") else args.steps
        r = run_form(w, p, k, args.warmup)
        r["steps"] = k
        log("form:", json.dumps(r))
        forms[p] = r
    del w
    sub = {}
    if args.sub:
        dims, sforms = args.sub.split(":")
        sx, sy, sz = (int(v) for v in dims.split("x"))
        ws = inputs.flume(nx=sx, ny=sy, nz=sz, seed=2)
        entry = {"spheres": ws.meta["spheres"], "cells": ws.ncells, "forms": {}}
        for p in [f for f in sforms.split(",") if f]:
            r = run_form(ws, p, args.sub_steps, args.warmup)
            r["steps"] = args.sub_steps
            log("sub form %s:" % ws.name, json.dumps(r))
            entry["forms"][p] = form_summary(r)
        sub[ws.name] = entry
        del ws
    copy_gbs = copy_bandwidth()
    log("device copy bandwidth %.0f GB/s" % copy_gbs)
    acc = None
    if not args.no_accuracy:
        weights = _WEIGHTS.get("w")
        if weights is None and main_res.get("estimator", {}).get("gate") is not None:
            weights = trained_estimator(fsl)[0]
        acc = accuracy_vs_oracle(weights)
    cpu = None if args.no_cpu else cpu_baseline(args.ny, args.nz)

    r = main_res
    base = args.precision.split("-")[0]
    name = "flume_%dx%dx%d" % (args.nx, args.ny, args.nz)
    traffic = stored_traffic(name, base)
    est = r.get("estimator")
    out = {
        "metric": "MLUPS free-surface D3Q27 cumulant (FP64/FP32/FP16-store), % HBM roofline",
        "value": r["mlups_fluid"], "unit": "MLUPS (fluid cells)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16-store/f32", "fp64": "f64"}[base],
        "data": "synthetic seeded flume (no dataset)",
        "config": {"workload": name, "precision": args.precision,
                   "estimator": ("finite differences" if not est else
                                 "learned with finite-difference fallback" if est["network_on"] else
                                 "learned, gated off (it does not beat finite differences in the flume's "
                                 "flow): finite differences in every cell"),
                   "estimator_gate": (est or {}).get("gate"),
                   "spheres": meta["spheres"], "depth": meta["depth"],
                   "cells": args.nx * args.ny * args.nz},
        "roofline": {"bound": "hbm", "achieved": r["bulk_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["bulk_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_bulk", "bytes_per_launch": r["bytes_per_launch"],
                     "pdf_only_achieved": r["bulk_pdf_gbs"],
                     "avg_launch_us": r["bulk_us"], "copy_gbs": copy_gbs,
                     "frac_of_copy": r["bulk_gbs"] / copy_gbs},
        "step_roofline": {"achieved": r["step_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": r["step_gbs"] / HBM_PEAK_GBS, "bytes_per_step": r["bytes_per_step"]},
        "cpu_baseline": cpu,
        "mlups_all_cells": r["mlups_all"],
        "mass_drift": r["mass_drift"],
        "forms": {k: form_summary(v) for k, v in forms.items()},
        "sub": sub,
        "accuracy_vs_oracle": acc,
        "wall_seconds": time.perf_counter() - t_start,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
