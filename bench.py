"""Benchmark of the free-surface cumulant LBM step on one MI355X.

One step = one pass of the whole hot path (dense stream-collide, interface
stream-collide with normals/curvature, reconstruction and mass flux,
conversion, excess mass) over the synthetic sediment flume 1536 x 40 x 192
(three layers of diameter-10 spheres with small prescribed velocities, 60
cells of liquid above the bed, FP32 PDF storage).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]

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


def learned_weights(lat, fsl, n_analytic=100000, steps=200, every=50, epochs=10, seed=0):
    """Train the estimator for a lattice: analytic stencils plus height-
    function labelled stencils of the lattice's own fill fields (taken while
    it runs the plain estimator), on the GPU; returns weights and report."""
    from paper_2301_10674_amd import train as T

    t0 = time.perf_counter()
    Xa, Ya = T.analytic_dataset(n_analytic, seed=seed)
    Xf, Yf = T.flume_dataset(lat, fsl, steps, every, n_analytic, seed=seed)
    X, Y = np.concatenate([Xa, Xf]), np.concatenate([Ya, Yf])
    Xt, Yt, Xv, Yv = T.split(X, Y, 0.1, seed=seed)
    rep = T.train(fsl, Xt, Yt, Xv, Yv, epochs=epochs, seed=seed)
    rep["data_seconds"] = time.perf_counter() - t0 - rep["train_seconds"]
    w = rep.pop("weights")
    rep.pop("losses")
    return w, rep


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


def run_form(w, form, steps, warmup, main_form=None):
    import torch

    from paper_2301_10674_amd import fsl

    precision, learned = form.split("-")[0], form.endswith("-learned")
    # "-variants": Thuerey's flux modifiers and normal-weighted excess mass,
    # curvature from corner normals
    variants = form.endswith("-variants")
    lat = fsl.lattice_from_workload(w, precision, normals=1 if learned else 0,
                                    flux_modifiers=variants, normal_excess=variants, csf_curvature=variants)
    est = None
    if learned:
        weights, est = learned_weights(lat, fsl)
        if est["gate"]:
            lat.set_estimator(weights)
    lat.step(warmup)
    torch.cuda.synchronize()
    liq0, itf0 = fluid_counts(lat, fsl)
    M0 = lat.total_mass()
    used0 = lat.estimator_stats() if learned else (0, 0)
    lat.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.timing(False)
    bulk_ms, launches = lat.timing_read()
    liq1, itf1 = fluid_counts(lat, fsl)
    M1 = lat.total_mass()
    secs = t1 - t0
    liq = 0.5 * (liq0 + liq1)
    fluid = 0.5 * (liq0 + itf0 + liq1 + itf1)
    s = STORE_BYTES[precision]
    bulk_avg_s = bulk_ms / 1e3 / max(launches, 1)
    bytes_per_launch = liq * (54 * s + 16) + w.ncells * 1
    # whole step: the dense pass plus the interface cells (own and pulled
    # PDFs read, PDFs written, fill level, mass, density, mark)
    itf = 0.5 * (itf0 + itf1)
    bytes_per_step = bytes_per_launch + itf * (81 * s + 44)
    res = dict(
        form=form, precision=precision, secs=secs, ms_per_step=1e3 * secs / steps,
        mlups_fluid=fluid * steps / secs / 1e6, mlups_all=w.ncells * steps / secs / 1e6,
        bulk_us=1e6 * bulk_avg_s, bulk_launches=launches,
        bulk_gbs=bytes_per_launch / bulk_avg_s / 1e9, bytes_per_launch=bytes_per_launch,
        step_gbs=bytes_per_step / (secs / steps) / 1e9, bytes_per_step=bytes_per_step,
        liquid_cells=liq, fluid_cells=fluid, interface_cells=0.5 * (itf0 + itf1),
        mass_drift=abs(M1 - M0) / M0, interface_error=interface_error(lat, fsl))
    if learned:
        used1 = lat.estimator_stats()
        res["estimator"] = dict(est, network_cells=used1[0] - used0[0], fallback_cells=used1[1] - used0[1])
    if len(w.radius) and form == main_form:
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


def cpu_baseline(seconds_target=12.0):
    """The FP64 oracle on the same flume recipe cropped to 128 x 40 x 192,
    for as many steps as fit in about seconds_target: once on one thread
    (the reported value) and once on all host threads (its per-cell phases
    run in parallel; the result does not depend on the thread count)."""
    from oracle import oracle as O
    from paper_2301_10674_amd import inputs

    w = inputs.flume_crop(nx=128, seed=3)

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
    O.set_threads(0)
    return {"value": v1, "unit": "MLUPS (fluid cells)", "cores": c1, "kind": "oracle",
            "sample": "FP64 oracle, flume recipe cropped to 128x40x192 (%d fluid cells), "
                      "%d steps after 1 warm-up step, %.1f s on 1 thread" % (fluid, n1, s1),
            "all_cores": {"value": va, "cores": ca,
                          "sample": "%d steps after 1 warm-up step, %.1f s on %d threads" % (na, sa, ca)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "fp64", "fp32-learned", "fp16-learned"])
    ap.add_argument("--nx", type=int, default=1536)
    ap.add_argument("--ny", type=int, default=40)
    ap.add_argument("--nz", type=int, default=192)
    ap.add_argument("--forms", default="fp16,fp64,fp32-learned,fp32-variants",
                    help="other forms timed on the same workload ('' for none): fp16, fp64, fp32, "
                         "fp32-learned (estimator trained in the run, see train.py), "
                         "fp32-variants (flux modifiers, normal-weighted excess mass, corner-normal curvature)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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

    fsl.lib()  # fails loudly if the HIP library is missing
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    log("building flume %dx%dx%d" % (args.nx, args.ny, args.nz))
    w = inputs.flume(nx=args.nx, ny=args.ny, nz=args.nz, seed=2)
    log("spheres %d, bed height %.2f, surface %.2f" % (w.meta["spheres"], w.meta["bed_height"],
                                                      w.meta["surface"]))
    main_res = run_form(w, args.precision, args.steps, args.warmup, main_form=args.precision)
    log("main form:", json.dumps(main_res))
    forms = {args.precision: main_res}
    for p in [f for f in args.forms.split(",") if f and f != args.precision]:
        r = run_form(w, p, max(args.steps // 2, 10), min(args.warmup, 20))
        log("form:", json.dumps(r))
        forms[p] = r
    copy_gbs = copy_bandwidth()
    log("device copy bandwidth %.0f GB/s" % copy_gbs)
    cpu = None if args.no_cpu else cpu_baseline()

    r = main_res
    base = args.precision.split("-")[0]
    traffic = stored_traffic(w.name, base)
    out = {
        "metric": "MLUPS free-surface D3Q27 cumulant (FP64/FP32/FP16-store), % HBM roofline",
        "value": r["mlups_fluid"], "unit": "MLUPS (fluid cells)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16-store/f32", "fp64": "f64"}[base],
        "data": "synthetic seeded flume (no dataset)",
        "config": {"workload": w.name, "precision": args.precision, "spheres": w.meta["spheres"],
                   "depth": w.meta["depth"], "cells": w.ncells},
        "roofline": {"bound": "hbm", "achieved": r["bulk_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["bulk_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_bulk", "bytes_per_launch": r["bytes_per_launch"],
                     "avg_launch_us": r["bulk_us"], "copy_gbs": copy_gbs,
                     "frac_of_copy": r["bulk_gbs"] / copy_gbs},
        "step_roofline": {"achieved": r["step_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": r["step_gbs"] / HBM_PEAK_GBS, "bytes_per_step": r["bytes_per_step"]},
        "cpu_baseline": cpu,
        "mlups_all_cells": r["mlups_all"],
        "mass_drift": r["mass_drift"],
        "forms": {k: {kk: v[kk] for kk in ("mlups_fluid", "ms_per_step", "bulk_gbs", "mass_drift",
                                          "interface_error", "estimator", "particle_forces_ms", "particles") if kk in v}
                  for k, v in forms.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
